"""tqr -- tiled QR factorisation (Buttari, Langou, Kurzak, Dongarra) for one
AMD MI355X (gfx950).

The compute path is the HIP library ``libtqr.so`` built from ``csrc/``;
``paper_0707_3548_amd.tqr`` is its ctypes binding.  Importing the package
does not load the library, so the input generators in ``workloads`` can be
used on machines without a GPU.
"""

__all__ = ["tqr", "workloads"]
