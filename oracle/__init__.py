"""Plain FP64 CPU oracle for the SO-FFT + ECS method of Serov & Sergeeva,
"Solution of the Schroedinger equation using exterior complex scaling and
fast Fourier transform" (arXiv:1505.06707).

THIS PACKAGE IS TEST INFRASTRUCTURE, NOT PART OF THE PRODUCT.  Only the test
suite, the smoke check of ``__graft_entry__`` and the ``cpu_baseline`` leg of
``bench.py`` may import it.  The HIP library never calls into it, and it shares
no code, tables or helpers with the HIP library: every formula here is written
out again from the paper.

The oracle is deliberately slow and literal:

* ``grid``    -- cell-centred DVR grid, momentum ordering and the unitary DFT
                 matrix F (Sec. II, Eqs. DVRgrid, DVRbasis, FFTbasis, Fmatrix).
* ``contour`` -- ECS contours q(x) and z(x) = int_0^x q (Sec. II Eq. ECSintdef;
                 Sec. IV sharp contour and smooth contour Eq. qSECS).
* ``ecs``     -- three-point K_s and K_FD, the remainder C = K_s - K_FD and the
                 Crank-Nicolson factor for exp(-i C tau) (Sec. II Eqs. C_FD,
                 Ks_FD, K_FD and the CN formula).
* ``tdse``    -- the split-operator step K/2 . U/2 . C . U/2 . K/2 applied
                 literally with four FFTs per step (Sec. II), 1D and 2D.
* ``sse``     -- the stationary matrix A = F^-1 K F + C + U - E (Sec. III
                 Eq. linsys), the FFT preconditioner (Eq. PreconFFT), COCG,
                 and a dense direct solve for tiny grids.
* ``learned`` -- FP64 forward/backward of the small periodic 3x3 convolution
                 network used as a correction to the FFT preconditioner, and
                 the flexible COCG that applies it (not from the paper).

Readings of the paper where it is silent or garbled are listed at the top of
each module.  Parity of every function is pinned by the ``-m "not gpu"`` tests
against closed forms, invariants and brute force.
"""
