"""MI355X (gfx950) Yukawa-FMM heat stepper after Kropinski & Quaife (arXiv 1007.5335).

The compute path is libyk.so (HIP kernels + C ABI, declared in include/yk.h);
`paper_1007_5335_amd.yk` is its thin ctypes binding.  Build with
`python -m paper_1007_5335_amd.build`.
"""
__all__ = ["yk", "build"]
