"""CPU oracle for the random-phase ensemble spin-dynamics path.

TEST INFRASTRUCTURE ONLY.  Only the test-suite, the smoke check and the
CPU-baseline leg of the benchmark may import anything under ``oracle/``.
The product path (the HIP library and its Python binding) never calls it,
and this package imports nothing from the product path.

Everything here is plain, slow and obviously correct: numpy / scipy in FP64,
or the plain C loop in ``trotter_ref.c``.  Each function states the passage
of Alvarez, Danieli, Levstein & Pastawski, "Quantum parallelism as a tool
for ensemble spin dynamics calculations" (arXiv:0710.3747) that it follows.

Conventions (readings of the paper, fixed for parity):
* site s (0-based; the paper's site 1 is site 0) is bit s of the basis
  index x; bit value 0 is spin up (I^z = +1/2);
* the random-phase state has amplitude exp(+i phi_r) / sqrt(2^(M-1)) on
  every basis state with the polarised site up, where r is x with that
  site's bit deleted and phi_r = 2 pi u(seed, r) (``phase.py``);
* one Trotter step is the symmetric (Strang) product: factors for the
  coupling list in list order with tau = dt/2, then in reverse order with
  tau = dt/2; each factor is exp(-i tau H_ij) exactly;
* P[k] = sum_x (1 - 2 bit_n'(x)) |psi_x|^2 after k steps (not divided by
  the norm); N[k] = sum_x |psi_x|^2.

Parity status of every function is listed in its module header.
"""
from .phase import splitmix64_next, phase_u, phase_u_array  # noqa: F401
from .state import (random_phase_state, random_phase_amplitudes, product_state,  # noqa: F401
                    product_phases)
from .trotter import (apply_factor, strang_factors, trotter_step,  # noqa: F401
                      trotter_run, trotter_profile, local_polarization, norm2)
from . import ed, sector  # noqa: F401
