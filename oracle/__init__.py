"""FP64 CPU oracle for the RPA polarizability band sum (TEST INFRASTRUCTURE ONLY).

This package is the independent reference that the GPU library is checked
against.  Only the test suite, the smoke check and the benchmark's CPU-baseline
leg may import it; the product path never does.  It shares no code with the HIP
library: plain NumPy/SciPy in float64/complex128, no blocking or fusion beyond
what the equations state.

Each function cites the passage of Gao, Xia, Gao & Zhang, "Towards Fully
Converged GW Calculations for Large Systems" (arXiv:1601.06767) it follows.
Readings taken where the paper is silent or garbled are listed in the module
docstrings that use them.

Pins (tests/test_oracle.py): every function here is checked against something
other than itself -- a brute-force plane-wave convolution, closed forms for
plane-wave states, orthogonality, Parseval, Hermiticity and sign of the static
polarizability, the exact band sum that the grouped form reduces to, the
printed speed-up tables, the free-electron state count, a Cholesky route for the
inverse, and central finite differences for every gradient.
"""
from .chi0 import (  # noqa: F401
    box_map, psi_real_space, pair_density_fft, pair_density_direct, weights, weights_static,
    chi0_from_pair_densities, chi0_bands, chi0_grouped_static, group_windows, group_edges, free_electron_dos,
    speedup_factor, alias_free,
)
from .dielectric import eps_matrix, eps_inv, eps_inv_static_cholesky, eps_inf  # noqa: F401
from .sigma import coh_kernel, sigma_coh_static, sigma_coh_complete_set, gpp_coh_kernel, sigma_coh_gpp  # noqa: F401
from .kpoints import kq_map, pair_density_kq, chi0_ksum, grad_chi0_ksum_energies  # noqa: F401
from .gpp import gpp_modes, gpp_eps_inv  # noqa: F401
from .grad import (  # noqa: F401
    grad_eps_inv, grad_weights_dynamic, grad_chi0_energies, head_block_loss,
)
