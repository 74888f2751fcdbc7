"""MI355X-native volume-averaged lattice Boltzmann solver (arXiv:1406.6438).

The hot path is a fused D2Q9 stream+collide sweep written in HIP for gfx950,
behind the C-ABI library ``liblbm_vans.so`` (declared in ``include/lbm_vans.h``).
``paper_1406_6438_amd.lbm`` is the thin ctypes binding; every step of the
method runs in the HIP kernels.  ``paper_1406_6438_amd.workloads`` holds the
seeded synthetic inputs.
"""
