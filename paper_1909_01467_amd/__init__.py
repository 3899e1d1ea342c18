"""L-sweeps GMRES for the PML-truncated Helmholtz equation on MI355X (gfx950).

The compute path is the C-ABI library ``liblsw.so`` (hand-written HIP kernels plus a
C++ host runtime); ``lsweeps`` is its thin ctypes binding.  ``inputs`` holds the seeded
synthetic workloads.
"""
