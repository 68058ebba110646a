"""MI355X-native rational-program fitting and launch-parameter selection.

The compute path is the C-ABI library ``librpfit.so`` (hand-written HIP for
gfx950, built in-tree).  ``paper_1906_00142_amd.rp`` is a thin ctypes binding
with the library's entry-point names; it loads the library on first use and
raises if it is missing.  ``paper_1906_00142_amd.workloads`` draws the seeded
synthetic inputs.
"""
__all__ = ["rp", "workloads"]
