"""FP64 CPU oracle for QMC-slicing kernel summation (Hertrich, Jahn,
Quellmalz, "Fast Summation of Radial Kernels via QMC Slicing", ICLR 2025).

TEST INFRASTRUCTURE ONLY.  This package is a plain, slow, obviously correct
reference written from the paper.  Only the test-suite, the smoke check of
``__graft_entry__`` and the ``cpu_baseline`` leg of ``bench.py`` may import
it.  The GPU library never imports, links or calls anything here, and nothing
here imports the GPU library: the two share no code.

Three references, each citing the passage it follows:
  O1  ``direct``   exact kernel sum, eq. (kernel_sum)               O(NMd)
                   (explicit differences, or the Gram identity for
                   large d)
  O2  ``sliced``   sliced sum with the exact 1-D basis function f,
                   eq. (kernel_sum_sliced)                          O(PNM)
  O3  ``fourier``  sliced sum with the truncated Fourier series of the
                   rescaled 1-D kernel summed as an exact non-uniform DFT,
                   App. I Steps 1-3 and eq. (Fourier-slicing)       O(P N_ft (N+M))
plus their analytic gradients.  Everything is float64.
"""
from .kernels import (KERNELS, basis_F, basis_dF, energy_cd, sliced_ft,
                      SlicedBasis, rescale_tau, fourier_coefficients,
                      truncated_coefficients)
from .direct import kernel_sum_direct, kernel_sum_direct_gram, grad_y_direct
from .sliced import kernel_sum_sliced, grad_sliced_energy
from .qmc import distance_energy, distance_energy_grad, projected_adam, rotate_directions
from .fourier import (kernel_sum_fourier, grad_y_fourier, grad_w_fourier, grad_x_fourier,
                      project)

__all__ = [
    "KERNELS", "basis_F", "basis_dF", "energy_cd", "sliced_ft", "SlicedBasis",
    "rescale_tau", "fourier_coefficients", "truncated_coefficients",
    "kernel_sum_direct", "kernel_sum_direct_gram", "grad_y_direct", "kernel_sum_sliced", "grad_sliced_energy",
    "kernel_sum_fourier", "grad_y_fourier", "grad_w_fourier", "grad_x_fourier", "project",
    "distance_energy", "distance_energy_grad", "projected_adam", "rotate_directions",
]
