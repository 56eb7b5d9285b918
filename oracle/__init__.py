"""Plain FP64 CPU oracle for the hPLMM preconditioned solve.

TEST INFRASTRUCTURE ONLY.  Nothing in the product path (the HIP library and
its Python binding) may import, call or link anything in this package.  Only
``tests/``, ``__graft_entry__.smoke()`` and the ``cpu_baseline`` leg of
``bench.py`` use it.

It is a slow, literal implementation written from the paper (Khan & Mehmani,
"High-order Multiscale Preconditioner for Elasticity of Arbitrary
Structures", arXiv 2509.19777):

* ``fem``        Sec. 2, Eqs. (1)-(4): Q1 voxel elasticity, assembly, loads.
* ``partition``  Sec. 3.1-3.2: grain grids, contact interfaces, contact grids.
* ``mortar``     Sec. 3.3, Eqs. (7)-(8): mortar nodes and Gaussian mortars.
* ``hplmm``      Sec. 4, Eqs. (16)-(26): W, Q, P, M_G, M_zeta, M_g, M_CG, M.
* ``gmres``      Sec. 5: right-preconditioned (and flexible) GMRES.
* ``precision``  rounding to FP32 / BF16 for the reduced-precision smoother.

Readings of passages the paper leaves open are listed in each module header
and in the design notes of the repository.
"""
