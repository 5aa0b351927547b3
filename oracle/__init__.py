"""Plain FP64 CPU oracle of the kernel-free boundary integral (KFBI) operator.

TEST INFRASTRUCTURE ONLY.  Only ``tests/``, ``__graft_entry__.smoke()`` and the
``cpu_baseline`` leg of ``bench.py`` may import this package.  The GPU library never calls
it, and it shares no code with the GPU library.

It follows the paper (Zhao, Dong, Ying, "Kernel free boundary integral method for 3D Stokes
and Navier equations on irregular domains") step by step, in numpy/scipy, slow and plain:

* geometry.py  -- grids (Sec. 4.2), level sets, crossings of the surface with grid lines,
                  control points and local frames (Algorithm 1 step 1).
* surface.py   -- least-squares surface derivatives of the density and the interface jump
                  relations (Sec. 4.2-4.3; the paper omits their derivation).
* mac.py       -- MAC operators, the sine-transform Poisson solver, the Schur-complement CG
                  (Sec. 4.2 items i-iii), the dense augmented solve for tiny grids, and the
                  irregular-node corrections (Sec. 4.3 cases 1-4).
* interp.py    -- the ten-node quadratic interpolation with jump function (Sec. 4.4).
* kfbi.py      -- the operator K phi = 1/2 phi - M phi, its transpose, GMRES and the
                  Dirichlet BVP (Sec. 3, Algorithm 1 steps 2-3).

Every reading of a silent or garbled passage is stated where it is used.
"""
