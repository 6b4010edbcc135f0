"""Plain FP64 CPU oracle for the voxel J-VIE hot path.

TEST INFRASTRUCTURE ONLY.  Nothing in the product path imports, calls, links or
executes this package; only the test-suite, the smoke check and the CPU-baseline
leg of the benchmark do.  It shares no code with the GPU library: the only
common module is the seeded input generator ``paper_1803_06237_amd.inputs``,
which holds none of the method's arithmetic.

Contents (each function cites the passage it follows):

* ``green``   -- Galerkin entries of the Green-tensor operator N on a uniform voxel
                grid (Section III-A): volume term V(m), face-face terms F^{ab}(m).
* ``fft``     -- the oracle's own FFT (iterative radix-2, Bluestein otherwise).
* ``matvec``  -- contrast chi, direct-sum and FFT matvec of ``I - M_eps N``,
                dense assembly (Section III-A; Section V-D).
* ``solve``   -- dense LU solve, GMRES(m) and flexible GMRES with CGS2 Arnoldi,
                brute-force Krylov minimum residual (Section V-D).
* ``observables`` -- field from currents and the reflection coefficient R (Section V-A).
* ``nn``      -- reference 3-D convolution forward/backward with BF16-rounded operands.
"""
