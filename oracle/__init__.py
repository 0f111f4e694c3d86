"""CPU oracle for the Sparse Bessel Decomposition (SBD) matvec.

TEST INFRASTRUCTURE ONLY.  Nothing in the product path may import, call or
execute this package: only ``tests/``, ``__graft_entry__.smoke()`` and the
``cpu_baseline`` leg of ``bench.py`` use it.  It shares no code with the GPU
library (``paper_1711_07877_amd``); the only common dependency is the seeded
input generator module ``synth``.

Everything here is plain, slow, FP64 numpy/scipy, written from the paper
(M. Averseng, "Fast discrete convolution in R^2 using Sparse Bessel
Decomposition"), following its notation:

* ``direct``    the discrete convolution itself (Introduction, eq.
                "discreteConv"), the exact definition the method approximates,
                and its two-set form (targets apart from sources, Section 7).
* ``sbd_fit``   Fourier-Bessel basis (Section 2.1), the SBD least-squares fit
                (Section 3.1, quadratic form Q^P; Section 3.2, eq.
                "LinearSystem" and the explicit Gram matrix A^P), the order
                search (Section 1, "Sparse Bessel Decomposition" paragraph),
                circle sizes M_p (Section 5, Theorem "QuadratureCirc" and
                eq. "temp1") and the weights (Section 6.2).
* ``sbd``       the whole off-line/on-line algorithm of Section 1 with the two
                NUFFTs replaced by exact exponential sums.
* ``nearfield`` the fixed-radius pair set and the close-correction matrix D
                (Section 1, eq. "defD"), both by the radial SBD series and by the
                paper's own assembly (an exponential sum over the circle nodes
                at the pair differences).
* ``binning``   the integer index build the GPU plan reports (cell keys, a
                stable sort, CSR rows), compared bit for bit.
* ``general``   the SBD of a general radial kernel with the multi-Dirichlet
                condition enforced by subtracting dilated J0 terms (Section 4.3).

Readings of the paper that the oracle takes (where it is silent, garbled or
inconsistent) are listed in the module docstrings where they apply.
"""
from .kernels import laplace_kernel, helmholtz_kernel
from .direct import direct_sum, direct_sum_targets, direct_sum_general, general_kernel_values
from .sbd_fit import (bessel_basis, gram_matrix, rhs_laplace, rhs_helmholtz, fit_coefficients,
                      choose_order, circle_sizes, SBDFit, fit_laplace, fit_helmholtz)
from .sbd import sbd_oracle, geometry, default_delta_min, frequencies
from .nearfield import near_pairs, near_values, near_values_nufft, near_pairs_targets, near_values_targets
from .binning import bin_keys, stable_perm, csr_from_perm

__all__ = [
    "laplace_kernel", "helmholtz_kernel", "direct_sum", "direct_sum_targets", "near_pairs_targets",
    "near_values_targets", "near_values_nufft", "frequencies", "bessel_basis", "gram_matrix",
    "rhs_laplace", "rhs_helmholtz", "fit_coefficients", "choose_order", "circle_sizes",
    "SBDFit", "fit_laplace", "fit_helmholtz", "sbd_oracle", "geometry", "default_delta_min",
    "near_pairs", "near_values", "bin_keys", "stable_perm", "csr_from_perm",
]
