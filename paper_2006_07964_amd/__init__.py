"""MI355X-native right-hand side + TVD-RK3 stage of a curvilinear high-order
finite-difference compressible Navier-Stokes solver (Ye et al., arXiv 2006.07964).

The compute path is the HIP library ``libcfd.so`` (sources in ``csrc/``, C ABI in
``include/cfd.h``); ``binding`` marshals arguments to it.  ``workloads`` builds seeded
synthetic grids and flow states.  Submodules are imported on demand so that the input
generators can be used without loading the GPU library.
"""
__all__ = ["binding", "workloads"]
