"""FP64 CPU oracle of the Tucker-compressed FFT-VIE matvec and solver.

TEST INFRASTRUCTURE ONLY.  Nothing in the product path may import or call
this package: only the tests, the smoke check and the CPU-baseline leg of the
benchmark use it.  It shares no code with the GPU library; both consume the
problem data built by ``vie_inputs``.

Everything is plain numpy / scipy in complex128, written to be checked by eye
against the paper (Giannakopoulos, Litsarev, Polimeridis, "Memory footprint
reduction for the FFT-based volume integral equation method via tensor
decompositions"):

* ``tucker``    -- unfoldings, n-mode products (App. I, Def. A.3), HOSVD
                   (Sec. IV-A, Alg. 1) and the Tucker model (Sec. III, eq. 13-14)
* ``circulant`` -- circulant embedding and Fourier-domain Tucker factors
                   (Sec. V-A)
* ``operator``  -- the electric block of the VIE operator (eq. 1-4, Sec. II-B):
                   brute-force Toeplitz sum, FFT convolution, Tucker matvec,
                   adjoint
* ``gmres``     -- restarted GMRES (Sec. VI-C solver settings)
* ``physics``   -- total field, absorbed power (eq. 18) and the Mie series
* ``gradient``  -- adjoint gradient of a field objective w.r.t. the per-voxel
                   permittivity and conductivity
* ``cp``        -- CP-ALS on the Tucker core and the Tucker+CP model
                   (Sec. IV-B, Alg. 2, eq. 15 and 17)
"""
