"""MI355X-native volume-averaged lattice Boltzmann solver (arXiv:1406.6438).

The hot path is a fused D2Q9 stream+collide sweep written in HIP for gfx950,
behind the C-ABI library ``liblbm_vans.so`` (declared in ``include/lbm_vans.h``).
``paper_1406_6438_amd.lbm`` is the thin ctypes binding; every step of the
method runs in the HIP kernels.  ``paper_1406_6438_amd.workloads`` holds the
seeded synthetic inputs.

Typical use (device memory and the stream come from torch)::

    import numpy as np
    from paper_1406_6438_amd import lbm

    p = lbm.Params(Lx=1024, Ly=512, tau=0.8, bc_x=lbm.BC_OPEN, bc_y=lbm.BC_BOUNCEBACK,
                   storage=lbm.F32_SHIFTED, d_p=20.0, u0=(0.02, 0.0),
                   rho_in=1.0, u_in=0.02, rho_out=1.0, u_out=0.02)
    eps = np.full((512, 1024), 0.7)          # porosity, one value per node
    s = lbm.Solver(p, eps)                   # on cuda:0
    s.step(1000)                             # asynchronous on torch's stream
    m = s.moments()                          # eps_rho, rho, ux, uy tensors + diagnostics
    J, dJdeps = s.grad(4000, ckpt_every=200) # outlet mass flux and its porosity gradient
    print(s.pass_plan)                       # (steps per pass, rows per chunk)
    s.close()

    # many independent problems advanced by batched launches
    sv = [lbm.Solver(q, e) for q, e in problems]
    b = lbm.Batch(sv)
    b.tune()                                 # pick the launch shape on this GPU
    b.step(2000)
"""
