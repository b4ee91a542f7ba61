"""Holstein-model DQMC sweeps on one MI355X (gfx950).

The compute path is libhq.so (HIP kernels behind the C ABI of include/hq.h);
paper_1905_07440_amd.hq is its ctypes binding.  Importing the package does not
load the library; hq.load() does, and fails loudly when it is not built.
"""
__all__ = ["hq", "build"]
