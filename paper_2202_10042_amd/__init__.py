"""FS-1 Sinkhorn for the Wasserstein-1 metric on a uniform 1-D grid (MI355X / gfx950).

The compute path is the C-ABI library ``libfs1.so`` (hand-written HIP kernels);
``paper_2202_10042_amd.fs1`` is its thin ctypes binding.  ``inputs`` holds the
seeded workload generators.  Nothing is imported eagerly so that the generators
can be used without loading the GPU library.
"""
__all__ = ["fs1", "inputs"]
