"""CPU FP64 oracle for the variational FFT homogenization solver.

TEST INFRASTRUCTURE ONLY.  This package is the plain, slow, independent
definition of what the GPU library computes.  Only the test suite, the smoke
check of the build entry point and the CPU-baseline leg of the benchmark may
import it; the product path (the HIP library and its Python binding) never
does, and shares no code with it.  The only code both sides consume is the
seeded input generation in ``synthetic``, which holds none of the method's
arithmetic.

Contents (each function cites the passage of Lucarini & Segurado,
arXiv:1806.10599, that it follows):

* ``dft``         dense separable DFT matrices (no FFT algorithm)
* ``projection``  Fourier frequencies (Eq. 18), continuous Ghat (Eq. 19),
                  discrete Ghat' from the rotated-centred derivative
                  (Eqs. 20-21), the linear map G(A) (Eqs. 10-11)
* ``crystal``     FCC slip systems, orientation matrices, cubic stiffness
* ``material``    crystal-plasticity return mapping (flow rule Eq. 22) with
                  its consistent tangent; isotropic St-Venant-Kirchhoff phase
* ``solver``      Newton-Raphson over increments with CG linear solves
                  (Eqs. 12-16), commit of internal variables, fatigue
                  indicator parameters (Eqs. 23-24), macro stress
* ``fips``        non-local (grain-averaged) indicators (Eq. 25)
* ``umat``        Appendix A conversion from a Jaumann-rate tangent to dP/dF
* ``conv``        circular 3-D convolution network of the learned warm start
                  (forward, backward, Adam) in FP64
* ``metrics``     the paper's error measures (Eqs. 29-31)

Parity status of every function is listed in its module header.
"""
