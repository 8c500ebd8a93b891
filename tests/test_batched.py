"""Batched factorisation (many independent problems in one launch).

GPU: every problem's factor (R, the tiled V and T) is bitwise the one the
single-problem path computes with the same tiling (both apply the same
operations to every tile in the same order), R matches the unblocked oracle
after sign normalisation, and a launch captured in a graph gives the eager
result on every replay.  CPU: the host plan's checks and offsets, and the
tile-size table / autotuner on a fake timer."""
import ctypes

import numpy as np
import pytest

import oracle
from paper_0707_3548_amd import autotune, tqr, workloads


def _plan(shapes, tiles, null_a=False, ibs=None):
    probs = (tqr.BatchProblem * max(len(shapes), 1))()
    for i, ((m, n), b) in enumerate(zip(shapes, tiles)):
        probs[i] = tqr.BatchProblem(m, n, max(1, m), 0 if null_a else 4096, 8192, b, 0 if ibs is None else ibs[i], 0)
    return tqr.lib().tqr_batch_plan(len(shapes), probs), probs


def test_plan_offsets_and_checks():
    nb, probs = _plan([(40, 17), (16, 16), (300, 2)], [16, 32, 64])
    assert nb > 256
    offs = [probs[i].work_offset for i in range(3)]
    assert offs[0] == 256 and all(o % 256 == 0 for o in offs) and offs == sorted(offs)
    # tiles + dense V copies of problem 0: p=3, q=2 tiles of 16x16 plus q diagonal blocks
    assert offs[1] - offs[0] == -(-((3 * 2 + 2) * 256 * 8) // 256) * 256
    assert _plan([(10, 20)], [16])[0] == -2          # m < n
    assert _plan([(40, 17)], [48])[0] == -2          # tile size
    assert _plan([(40, 17)], [256])[0] == -2
    assert _plan([(40, 17)], [16], null_a=True)[0] == -2
    assert _plan([(40, 17)], [16], ibs=[32])[0] == -2    # inner block larger than the tile
    assert _plan([(40, 17)], [128], ibs=[64])[0] == -2   # panel too large for the chip
    assert b"problem 0" in tqr.lib().tqr_last_error_string()
    assert _plan([(40, 17), (70, 70)], [64, 32], ibs=[64, 32])[0] > 256
    assert tqr.lib().tqr_batch_plan(-1, None) == -1
    assert tqr.lib().tqr_batch_plan(0, None) == 256


def test_factor_batched_argument_checks():
    L = tqr.lib()
    fake = ctypes.c_void_p(64)
    assert L.tqr_factor_batched(-1, None, None, 0, None, 0, 0, None) == -1
    assert L.tqr_factor_batched(3, None, fake, 4096, None, 0, 0, None) == -2
    assert L.tqr_factor_batched(3, fake, None, 4096, None, 0, 0, None) == -3
    assert L.tqr_factor_batched(3, fake, fake, 100, None, 0, 0, None) == -4
    assert L.tqr_factor_batched(3, fake, fake, 4096, None, -1, 0, None) == -6
    assert L.tqr_factor_batched(3, fake, fake, 4096, None, 0, 7, None) == -7


def test_tile_table_and_tuner():
    assert autotune.tile_for(8) == 16 and autotune.tile_for(40) == 32 and autotune.tile_for(500) == 64
    assert autotune.tiling_for(500) == (64, 16)
    # older two-element tables mean inner block 16
    assert autotune.tiling_for(100, [(0, 32), (64, 128)]) == (128, 16)
    # a fake device where (32, 16) is fastest below n = 64 and (64, 32) above
    def sample(lo, hi):
        return [(max(16, lo + 1), lo + 1)] if lo < 512 else []

    def time_batch(shapes, b, ib):
        n = shapes[0][1]
        if n < 64:
            return 1.0 if (b, ib) == (32, 16) else 2.0 + b / 64 + ib / 64
        return 1.0 if (b, ib) == (64, 32) else 2.0 + b / 64 + ib / 64

    table = autotune.tune(sample, time_batch)
    assert table == [(0, 32, 16), (64, 64, 32)]
    assert autotune.tiling_for(10, table) == (32, 16) and autotune.tiling_for(100, table) == (64, 32)


def _torch():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    return torch


EDGE = [(16, 16), (16, 8), (17, 1), (64, 64), (65, 64), (100, 33), (512, 512), (300, 299), (40, 40), (33, 32)]


@pytest.mark.gpu
def test_batched_matches_single_problem_path():
    torch = _torch()
    shapes = workloads.batch_shapes(48, seed=5) + EDGE
    tiles = [autotune.tile_for(n) for _, n in shapes]
    tiles[-3:] = [16, 32, 64]
    print(f"case batched vs single: {len(shapes)} problems", flush=True)
    mats = workloads.batch_matrices(shapes, seed=6)
    bt = tqr.Batch(shapes, tiles)
    bt.load(mats)
    bt.factor()
    torch.cuda.synchronize()
    assert int(bt.status.item()) == 0
    for i, ((m, n), b) in enumerate(zip(shapes, tiles)):
        dA = tqr.fortran(torch.from_numpy(mats[i]).cuda())
        ws = tqr.Workspace(m, n, 0, b, 16)
        tqr.factor(dA, b, 16, ws)
        torch.cuda.synchronize()
        assert torch.equal(bt.matrix(i), dA), f"problem {i} ({m}x{n}, b={b}): factor differs"
        assert torch.equal(bt.t_slots(i), ws.T[:bt.t_slots(i).numel()]), f"problem {i}: T differs"


@pytest.mark.gpu
def test_batched_r_matches_oracle():
    torch = _torch()
    shapes = workloads.batch_shapes(200, seed=7)
    tiles = [autotune.tile_for(n) for _, n in shapes]
    print(f"case batched vs oracle: {len(shapes)} problems", flush=True)
    mats = workloads.batch_matrices(shapes, seed=8)
    bt = tqr.Batch(shapes, tiles)
    bt.load(mats)
    bt.factor()
    torch.cuda.synchronize()
    for i in range(0, len(shapes), 7):
        m, n = shapes[i]
        R = np.triu(bt.matrix(i).cpu().numpy()[:n, :])
        _, R_or = oracle.qr(mats[i])
        assert oracle.rel_fro(oracle.sign_normalize(R), R_or) < 1e-10, (i, m, n)


@pytest.mark.gpu
def test_batched_graph_replays_match_eager():
    torch = _torch()
    shapes = workloads.batch_shapes(300, seed=9)
    tiles = [autotune.tile_for(n) for _, n in shapes]
    print("case batched graph replay: 300 problems", flush=True)
    mats = workloads.batch_matrices(shapes, seed=10)
    bt = tqr.Batch(shapes, tiles)
    bt.load(mats)
    pristine = bt.A.clone()
    bt.factor()
    torch.cuda.synchronize()
    eager_A, eager_T = bt.A.clone(), bt.T.clone()
    s = torch.cuda.Stream()
    g = torch.cuda.CUDAGraph()
    bt.A.copy_(pristine)
    torch.cuda.synchronize()
    with torch.cuda.graph(g, stream=s):
        bt.factor()
    for rep in range(3):
        bt.A.copy_(pristine)
        bt.T.zero_()
        torch.cuda.synchronize()
        g.replay()
        torch.cuda.synchronize()
        assert torch.equal(bt.A, eager_A), f"replay {rep}: A differs"
        assert torch.equal(bt.T, eager_T), f"replay {rep}: T differs"
        assert int(bt.status.item()) == 0


@pytest.mark.gpu
@pytest.mark.parametrize("precision", ["fp64", "fp32"])
def test_batched_tuned_table_matches_single_path_and_oracle(precision):
    """The tilings the benchmark uses (autotune.current_table(), b = 128 for
    the widest problems), FP64 and FP32-update batches: every problem bitwise
    the single-problem path with the same tiling and precision, and R against
    the oracle (FP64: 1e-10; FP32 updates: FP32 accuracy, 1e-4)."""
    torch = _torch()
    prec = tqr.PRECISION_FP64 if precision == "fp64" else tqr.PRECISION_FP32_UPDATES
    table = autotune.current_table(precision)
    shapes = workloads.batch_shapes(160, seed=13) + [(512, 512), (500, 300), (300, 129), (257, 64), (130, 128)]
    tilings = [autotune.tiling_for(n, table) for _, n in shapes]
    tiles, ibs = [t[0] for t in tilings], [t[1] for t in tilings]
    print(f"case batched tuned table {precision} {table}: {len(shapes)} problems, tilings {sorted(set(tilings))}",
          flush=True)
    mats = workloads.batch_matrices(shapes, seed=14)
    bt = tqr.Batch(shapes, tiles, ibs, precision=prec)
    bt.load(mats)
    bt.factor()
    torch.cuda.synchronize()
    assert int(bt.status.item()) == 0
    for i, ((m, n), b, ib) in enumerate(zip(shapes, tiles, ibs)):
        dA = tqr.fortran(torch.from_numpy(mats[i]).cuda())
        ws = tqr.Workspace(m, n, 0, b, ib)
        tqr.factor(dA, b, ib, ws, precision=prec)
        torch.cuda.synchronize()
        assert torch.equal(bt.matrix(i), dA), f"problem {i} ({m}x{n}, b={b}, ib={ib}): factor differs"
        assert torch.equal(bt.t_slots(i), ws.T[:bt.t_slots(i).numel()]), f"problem {i}: T differs"
        if i % 5 == 0 or b >= 128:
            R = np.triu(bt.matrix(i).cpu().numpy()[:n, :])
            _, R_or = oracle.qr(mats[i])
            tol = 1e-10 if precision == "fp64" else 1e-4
            assert oracle.rel_fro(oracle.sign_normalize(R), R_or) < tol, (i, m, n, b, ib)


@pytest.mark.gpu
@pytest.mark.parametrize("precision", ["fp64", "fp32"])
def test_batched_every_tiling_matches_single_path(precision):
    """Every supported (tile_b, inner_ib) pair in one batch (FP32 updates:
    inner block 16 only; other pairs are reported through the status word
    and left untouched)."""
    torch = _torch()
    prec = tqr.PRECISION_FP64 if precision == "fp64" else tqr.PRECISION_FP32_UPDATES
    pairs = list(autotune.CANDIDATES)
    shapes, tilings = [], []
    for k, (b, ib) in enumerate(pairs):
        for (m, n) in ((3 * b + 5, 2 * b + 3), (b, b), (70 + 11 * k, 37 + 5 * k)):
            shapes.append((m, n))
            tilings.append((b, ib))
    ok_pairs = set(autotune.CANDIDATES_FP32) if precision == "fp32" else set(pairs)
    run = [i for i, t in enumerate(tilings) if t in ok_pairs]
    print(f"case batched every tiling {precision}: {len(run)} problems", flush=True)
    shapes = [shapes[i] for i in run]
    tilings = [tilings[i] for i in run]
    mats = workloads.batch_matrices(shapes, seed=15)
    bt = tqr.Batch(shapes, [t[0] for t in tilings], [t[1] for t in tilings], precision=prec)
    bt.load(mats)
    bt.factor()
    torch.cuda.synchronize()
    assert int(bt.status.item()) == 0
    for i, ((m, n), (b, ib)) in enumerate(zip(shapes, tilings)):
        dA = tqr.fortran(torch.from_numpy(mats[i]).cuda())
        ws = tqr.Workspace(m, n, 0, b, ib)
        tqr.factor(dA, b, ib, ws, precision=prec)
        torch.cuda.synchronize()
        assert torch.equal(bt.matrix(i), dA), f"problem {i} ({m}x{n}, b={b}, ib={ib}): factor differs"
    if precision == "fp32":
        # a pair the FP32 tier does not run is reported and skipped
        bad = tqr.Batch([(100, 70)], [64], [32], precision=prec)
        bad.load([workloads.gaussian(100, 70, seed=16)])
        before = bad.A.clone()
        bad.factor()
        torch.cuda.synchronize()
        assert int(bad.status.item()) == 1
        assert torch.equal(bad.A, before)
