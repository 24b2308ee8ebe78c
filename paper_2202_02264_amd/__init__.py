"""dSMC (de-Sequentialized Monte Carlo) particle smoother on AMD MI355X.

The HIP kernels and the C ABI live in ``libdsmc.so`` (sources in ``csrc/``,
header ``include/dsmc.h``); ``paper_2202_02264_amd.dsmc`` is the ctypes
binding.  ``workloads`` builds seeded synthetic models.  Submodules are
imported on demand so that ``workloads`` can be used without the GPU library.
"""
__all__ = ["dsmc", "workloads"]
