"""Seeded synthetic inputs shared by the oracle tests, the GPU parity tests and the
benchmark.  This module draws random numbers and lays them out; it holds none of the
method's arithmetic.

Every array comes from numpy ``Generator(PCG64(SeedSequence([180206177, config, item,
variant])))``, so any single item can be regenerated on its own (the parity tests sample
items of the full-size workloads one by one).

Workloads (shapes of the paper's simulations: square lattices L x L with L up to 20,
dtau = 0.1, beta = Ltau dtau; SM Eq. S1 and main text):

  W1  4x4,   Ltau=40,  n_s=10, lam=1.5: 48 Gaussian fields N(0, 1/sqrt(omega0)) and 16
      staggered CDW fields +-x0 (-1)^(ix+iy) + N(0, 0.1), x0 = lam/omega0^2 (items 48-55
      take +x0, 56-63 take -x0), static in time.
  W2  8x8,   Ltau=80,  n_s=10, lam=1.5: 256 Gaussian fields.
  W3  12x12, Ltau=120, n_s=10, lam=1.5: 64 chains, Gaussian initial fields, effective
      model coefficients drawn uniformly in [-0.5, 0.5].
  W4  16x16, Ltau=160, n_s=8, lam in {1.0, 1.5, 2.0}: 128 Gaussian fields per lam, plus
      16 staggered fields (x0 = lam/omega0^2).
  W5  uneven batch: 32 fields for each L in {8, 12, 16, 20}, beta = L, Ltau = 10 L,
      n_s = 10.
"""

from .fields import (
    gen, gaussian_field, cdw_field, workload_models, workload_fields, workload_item,
    eff_coefficients, physical_eff, WORKLOADS,
)

__all__ = [
    "gen", "gaussian_field", "cdw_field", "workload_models", "workload_fields",
    "workload_item", "eff_coefficients", "physical_eff", "WORKLOADS",
]
