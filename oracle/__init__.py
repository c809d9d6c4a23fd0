"""Plain, slow FP64 CPU oracle for the fermion weight of the Holstein model and the
symmetric-effective-model SLMC steps that use it.

TEST INFRASTRUCTURE ONLY.  Nothing in the product path may import, call or run this
package: only ``tests/``, ``__graft_entry__.smoke()`` and the ``cpu_baseline`` leg of
``bench.py`` use it.  It shares no code with the HIP library (no kernels, headers,
helpers, tables or constant generators) and it never imports the product package.

Every function cites the passage of arXiv:1802.06177 it follows (main text equations,
Supplemental Material equations S1-S8, Table S1).  Where the paper is silent or its
text is garbled, the reading taken is named in the docstring (labels A1..A26 are
listed with their justification in the design notes at the repository root).

Modules
-------
lattice    hopping matrix K and its exponential e^{-dtau K}          (SM Eq. S1)
fermion    stabilized product chain, log|det(1+B_L...B_1)|, sign, G (SM Eqs. S2, S3)
boson      bosonic action S_Bose and the full log-weight             (SM Eq. S2)
effective  symmetric effective model E_eff, local dE, checkerboard
           Metropolis sweep                                         (Eq. 4 / S7)
philox     Philox4x32-10 counter-based generator (Salmon et al., SC'11)
accept     SLMC cumulative-update acceptance                        (Eq. 6)
wolff      modified Wolff cluster moves and the cumulative proposal (SM Sec. IV, Eq. S8)
measure    G at every time slice and the CDW structure factor's estimators (SM Eq. S3)
dqmc       DQMC comparison updates: local ratio, Sherman-Morrison, block update (SM Sec. I)
train      effective-model features and their regression onto ln w (Eq. 5, SM Sec. III)
"""

from .lattice import hopping_matrix, expk
from .fermion import slice_scales, udv_chain, recombine, logdet_green, logdet_green_direct
from .boson import bosonic_action, log_weight
from .effective import EffModel, eff_energy, eff_local_delta, colouring, sweep
from .philox import philox4x32_10, uniform01
from .accept import cumulative_accept
from .wolff import cluster as wolff_cluster, wolff, propose
from .measure import green_slices, cdw_estimators, stagger
from .dqmc import local_ratio, sherman_morrison, local_sweep, block_updates
from .train import features as eff_features, fit as eff_fit, TERMS

__all__ = [
    "hopping_matrix", "expk", "slice_scales", "udv_chain", "recombine", "logdet_green",
    "logdet_green_direct", "bosonic_action", "log_weight", "EffModel", "eff_energy",
    "eff_local_delta", "colouring", "sweep", "philox4x32_10", "uniform01", "cumulative_accept",
    "wolff_cluster", "wolff", "propose", "green_slices", "cdw_estimators", "stagger",
    "local_ratio", "sherman_morrison", "local_sweep", "block_updates", "eff_features", "eff_fit",
    "TERMS",
]
