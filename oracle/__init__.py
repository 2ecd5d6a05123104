"""CPU FP64 oracle for the spherical Gauss-Laguerre (SGL) transform pair.

TEST INFRASTRUCTURE ONLY.  Only the test-suite, the package smoke check and the
CPU-baseline leg of the benchmark may import or call anything in this package.
The GPU library never links, imports or calls it, and this package never
imports the GPU library: the two share no code.

What it computes is the plain definition of the method: the quadrature sum of
the SGL sampling theorem (Thm. 3.4, Eq. SGL-Sampling-Theorem) for the forward
transform and the direct synthesis sum of the naive inverse (Alg. 2) for the
inverse, with every basis function evaluated point by point from its own
recurrences (Sect. 2) and the quadrature rules built from their definitions
(Thm. 3.1, Thm. 3.3).

Modules
-------
quadrature  equiangular S^2 rule (Thm. 3.1) and half-range Gauss-Hermite rule
            (Thm. 3.3), from moments in multiple precision.
basis       normalized associated Legendre functions (Def. 2.1, Eq.
            legendre_recurrence) and normalized radial functions (Def. 1.2,
            Eq. laguerre_recursion).
direct      the direct forward (Alg. 1) and inverse (Alg. 2) sums, full and on
            seeded subsets.
mp_direct   a 50-digit mpmath evaluation of Alg. 1/2 for tiny bandlimits, used
            to pin the FP64 oracle.

Readings of the paper taken here (each is pinned by a test):
  * the S^2 weight carries the azimuthal step pi/B (b~_j = (pi/B) b_j);
  * samples may be given "scaled", s_ijk = sigma_i f(r_i, th_j, ph_k) with
    sigma_i = sqrt(a_i) r_i, so that no value leaves the FP64 range;
  * the forward FFT uses exp(-i m phi_k), the inverse exp(+i m phi_k).
"""

from . import quadrature, basis, direct  # noqa: F401,E402

__all__ = ["quadrature", "basis", "direct"]
