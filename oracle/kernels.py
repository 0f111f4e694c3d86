"""Green's kernels of the paper (FP64).

* Laplace single layer G(x) = -(1/2 pi) log|x| (Introduction, after eq.
  "discreteConv").  Evaluated from the squared distance d2 as
  -(1/4 pi) log(d2) so that no square root is taken.
* Helmholtz G(x) = (i/4) H_0^(1)(k|x|) (Section 4.2 defines H^(1) = J0 + i Y0;
  the paper writes the kernel with a -i/4 prefactor, the workloads here use
  +i/4, which only flips the sign of the result).  H_0^(1) comes from
  ``scipy.special.hankel1``.
"""
import numpy as np
import scipy.special as sp


def laplace_kernel(d2):
    """-(1/(4 pi)) log(d2) for squared distances d2 > 0."""
    return -(1.0 / (4.0 * np.pi)) * np.log(d2)


def helmholtz_kernel(d2, k):
    """(i/4) H0^(1)(k sqrt(d2)) for squared distances d2 > 0."""
    return 0.25j * sp.hankel1(0, k * np.sqrt(d2))
