"""CPU FP64 oracle for the fast spin spherical-harmonic transform.

TEST INFRASTRUCTURE ONLY.  Nothing in the product path may import or call this
package: only ``tests/``, ``__graft_entry__.smoke()`` and the ``cpu_baseline``
leg of ``bench.py`` use it.  It shares no code with the HIP path.

What it computes (McEwen, "Fast, exact (but unstable) spin spherical harmonic
transforms", arXiv:0807.4494):

* :mod:`oracle.wigner` -- Delta^l_{m'm} = d^l_{m'm}(pi/2) for all m', m by
  Risbo's recursion (Section 2.2 names it; the half-step form is derived from
  the SU(2) polynomial model, see that module).
* :mod:`oracle.transform` -- the inverse transform through the torus Fourier
  coefficients of Eq. (fourier_coeff) and the 2-D Fourier sum of
  Eq. (sht_inv_fast); the forward transform as the exact quadrature of
  Eq. (ssht_fwd) on the periodically extended torus (Sections 3.2, 3.4.1).
* :mod:`oracle.metrics` -- the five error metrics of Section 4.2.
* :mod:`oracle.triangular` -- the paper's own forward transform (per-order
  triangular systems, Section 3.4.2), its least-squares variant and the
  stability experiment of Section 4.2.

Everything is float64 / complex128.  Pins (tests that tie each function to
something other than itself) live in ``tests/test_oracle_*.py``.
"""

from .wigner import delta_planes, delta_plane, DeltaRisbo
from .transform import (inverse, forward, fourier_coefficients, torus_synthesis,
                        theta_nodes, phi_nodes, quadrature_weight, inverse_batch,
                        forward_batch, forward_rows)
from .metrics import error_metrics, rel_l2
from . import triangular

__all__ = ["delta_planes", "delta_plane", "DeltaRisbo", "inverse", "forward",
           "fourier_coefficients", "torus_synthesis", "theta_nodes", "phi_nodes",
           "quadrature_weight", "inverse_batch", "forward_batch", "forward_rows",
           "error_metrics", "rel_l2"]
