"""Pins of the tiled model (Algorithm 1 run sequentially in numpy), the
reference for the V and T tiles.  The unblocked oracle fixes R; the compact
WY identity, built from explicit reflector products, fixes T; the single-tile
case fixes V against the unblocked reflectors.  CPU only."""
import numpy as np
import pytest

import oracle
from oracle import tiled
from paper_0707_3548_amd import workloads

EPS = oracle.EPS


def _reflector(v_full, tau):
    return np.eye(len(v_full)) - tau * np.outer(v_full, v_full)


@pytest.mark.parametrize("m,n,b,ib", [(512, 512, 64, 16), (200, 130, 64, 16), (97, 97, 32, 8),
                                      (130, 70, 64, 64), (7, 5, 1, 1), (300, 40, 16, 4), (256, 256, 128, 32)])
def test_r_matches_unblocked_oracle(m, n, b, ib):
    A = workloads.gaussian(m, n, seed=m * 7 + n)
    tiles, T = tiled.factor(A, b, ib)
    _, R_or = oracle.qr(A)
    R = oracle.sign_normalize(tiled.r_factor(tiles, m, n))
    assert oracle.rel_fro(R, R_or) < 1e-12
    Q = tiled.form_q(tiles, T, m, n)
    Rraw = tiled.r_factor(tiles, m, n)
    assert oracle.fact_error(A, Q, Rraw) <= 10 * n * EPS
    assert oracle.orth_error(Q) <= 10 * n * EPS


def test_single_tile_reflectors_equal_unblocked():
    """p = q = 1: the blocked GEQRT produces the same reflectors as DGEQR2;
    blocking only changes how they are applied."""
    b, ib = 64, 16
    A = workloads.gaussian(b, b, seed=21)
    tiles, T = tiled.factor(A, b, ib)
    P, tau = oracle.geqr2(A)
    V_t = np.tril(tiles[0, 0], -1)
    V_o = np.tril(P, -1)
    assert np.abs(V_t - V_o).max() < 1e-12
    tau_t = np.concatenate([np.diag(T[0, 0][:, s * ib:(s + 1) * ib]) for s in range(b // ib)])
    assert np.abs(tau_t - tau).max() < 1e-13
    assert np.abs(np.triu(tiles[0, 0]) - np.triu(P)).max() < 1e-12


def test_geqrt_compact_wy_identity():
    """I - V_s T_s V_s^T = H_{c0} H_{c0+1} ... H_{c0+ib-1}, with each H built
    explicitly from its vector and scalar."""
    b, ib = 32, 8
    A = workloads.gaussian(b, b, seed=22)
    Akk = A.copy()
    T = tiled.geqrt(Akk, ib)
    for c0 in range(0, b, ib):
        H = np.eye(b)
        Vs = np.zeros((b, ib))
        for jj in range(ib):
            j = c0 + jj
            v = np.zeros(b)
            v[j] = 1.0
            v[j + 1:] = Akk[j + 1:, j]
            Vs[:, jj] = v
            H = H @ _reflector(v, T[jj, j])
        Ts = T[:, c0:c0 + ib]
        assert np.allclose(np.tril(Ts, -1), 0)
        assert np.abs(np.eye(b) - Vs @ Ts @ Vs.T - H).max() < 1e-13


def test_tsqrt_compact_wy_identity():
    """Same identity for the stacked reflectors [e_j; v_j] of DTSQT2."""
    b, ib = 24, 6
    R = np.triu(workloads.gaussian(b, b, seed=23))
    A = workloads.gaussian(b, b, seed=24)
    Rk, Ak = R.copy(), A.copy()
    T = tiled.tsqrt(Rk, Ak, ib)
    for c0 in range(0, b, ib):
        H = np.eye(2 * b)
        Vs = np.zeros((2 * b, ib))
        for jj in range(ib):
            j = c0 + jj
            v = np.zeros(2 * b)
            v[j] = 1.0
            v[b:] = Ak[:, j]
            Vs[:, jj] = v
            H = H @ _reflector(v, T[jj, j])
        Ts = T[:, c0:c0 + ib]
        assert np.abs(np.eye(2 * b) - Vs @ Ts @ Vs.T - H).max() < 1e-13
    # and the stacked pair is factorised: [R; A] = Q [R~; 0]
    _, R_or = oracle.qr(np.vstack([R, A]))
    assert oracle.rel_fro(oracle.sign_normalize(np.triu(Rk)), R_or) < 1e-13


def test_tsqrt_leaves_strict_lower_part_alone():
    b, ib = 16, 4
    Akk = workloads.gaussian(b, b, seed=25)
    lower = np.tril(Akk, -1).copy()
    tiled.tsqrt(Akk, workloads.gaussian(b, b, seed=26), ib)
    assert np.array_equal(np.tril(Akk, -1), lower)


@pytest.mark.parametrize("b,ib", [(64, 16), (64, 64), (128, 32), (32, 8), (16, 16), (1, 1)])
def test_invariant_to_tiling(b, ib):
    A = workloads.gaussian(150, 120, seed=27)
    tiles, _ = tiled.factor(A, b, ib)
    _, R_or = oracle.qr(A)
    assert oracle.rel_fro(oracle.sign_normalize(tiled.r_factor(tiles, 150, 120)), R_or) < 1e-12


def test_apply_qt_of_a_is_r_and_apply_q_inverts():
    A = workloads.gaussian(200, 100, seed=28)
    tiles, T = tiled.factor(A, 32, 8)
    C = tiled.apply_qt(tiles, T, A)
    R = tiled.r_factor(tiles, 200, 100)
    assert np.abs(C[100:]).max() < 1e-12
    assert np.abs(np.triu(C[:100]) - R).max() < 1e-12
    B = workloads.gaussian(200, 3, seed=29)
    assert oracle.rel_fro(tiled.apply_q(tiles, T, tiled.apply_qt(tiles, T, B)), B) < 1e-14


def test_upper_triangular_input_exact():
    U = np.triu(workloads.gaussian(96, 96, seed=30))
    tiles, T = tiled.factor(U, 32, 8)
    assert np.array_equal(tiled.from_tiles(tiles, 96, 96), U)
    assert np.all(T == 0)


def test_padding_is_exact_zero():
    """Ragged edges: padded rows keep exactly zero reflector entries."""
    m, n, b = 100, 70, 32
    tiles, _ = tiled.factor(workloads.gaussian(m, n, seed=31), b, 8)
    full = tiles.transpose(0, 2, 1, 3).reshape(tiles.shape[0] * b, tiles.shape[1] * b)
    assert np.all(full[m:, :] == 0)
