"""Seeded phonon fields, model descriptions and effective-model coefficients."""

import numpy as np

ROOT_SEED = 180206177

# Lattice/Trotter parameters of the workloads (t = 1, mu = 0 in the build frame,
# omega0 = 1, dtau = 0.1, c_kin = 1/2 unless stated).
WORKLOADS = {
    "W1": dict(L=[4], Ltau=[40], n_s=10, lam=[1.5], items=64),
    "W2": dict(L=[8], Ltau=[80], n_s=10, lam=[1.5], items=256),
    "W3": dict(L=[12], Ltau=[120], n_s=10, lam=[1.5], items=64),
    "W4": dict(L=[16], Ltau=[160], n_s=8, lam=[1.0, 1.5, 2.0], items=128),
    "W5": dict(L=[8, 12, 16, 20], Ltau=[80, 120, 160, 200], n_s=10, lam=[1.5], items=128),
}
_CFG_ID = {"W1": 1, "W2": 2, "W3": 3, "W4": 4, "W5": 5}


def gen(config, item, variant=0):
    """Independent PCG64 stream for one (workload, item, variant)."""
    return np.random.Generator(np.random.PCG64(np.random.SeedSequence(
        [ROOT_SEED, int(config), int(item), int(variant)])))


def gaussian_field(g, Ltau, N, sigma):
    """x[l, i] i.i.d. normal with standard deviation sigma (reading A20)."""
    return g.normal(0.0, sigma, size=(Ltau, N))


def cdw_field(g, Lx, Ly, Ltau, x0, noise):
    """Static staggered field x0 (-1)^(ix+iy) plus i.i.d. N(0, noise) per (i, l)."""
    ix = np.arange(Lx * Ly) % Lx
    iy = np.arange(Lx * Ly) // Lx
    stag = np.where((ix + iy) % 2 == 0, 1.0, -1.0)
    return np.tile(x0 * stag, (Ltau, 1)) + g.normal(0.0, noise, size=(Ltau, Lx * Ly))


def model_dict(L, Ltau, n_s, lam, t=1.0, mu=0.0, dtau=0.1, omega0=1.0, c_kin=0.5):
    return dict(Lx=L, Ly=L, Ltau=Ltau, n_s=n_s, t=t, mu=mu, dtau=dtau, lam=lam,
                omega0=omega0, c_kin=c_kin)


def workload_models(name, lam_idx=0):
    w = WORKLOADS[name]
    lam = w["lam"][lam_idx]
    return [model_dict(L, Lt, w["n_s"], lam) for L, Lt in zip(w["L"], w["Ltau"])]


def workload_item(name, item, lam_idx=0):
    """(model_index, x[Ltau, N]) of one item of a workload."""
    w = WORKLOADS[name]
    c = _CFG_ID[name]
    lam = w["lam"][lam_idx]
    omega0 = 1.0
    if name == "W5":
        mi = item // 32
        L, Lt = w["L"][mi], w["Ltau"][mi]
    else:
        mi, L, Lt = 0, w["L"][0], w["Ltau"][0]
    N = L * L
    g = gen(c, item, lam_idx)
    if name == "W1" and item >= 48:
        x0 = lam / omega0 ** 2
        sgn = 1.0 if item < 56 else -1.0
        return mi, cdw_field(g, L, L, Lt, sgn * x0, 0.1)
    if name == "W4" and item >= w["items"]:
        # the 16 extra staggered fields of W4 (closed-form check), noiseless
        x0 = lam / omega0 ** 2
        sgn = 1.0 if (item - w["items"]) % 2 == 0 else -1.0
        return mi, cdw_field(g, L, L, Lt, sgn * x0, 0.0)
    return mi, gaussian_field(g, Lt, N, 1.0 / np.sqrt(omega0))


def workload_fields(name, n_items=None, lam_idx=0):
    """List of (model_index, x) for the first n_items items of a workload."""
    n = WORKLOADS[name]["items"] if n_items is None else n_items
    return [workload_item(name, b, lam_idx) for b in range(n)]


def eff_coefficients(config, variant, lam, omega0=1.0, delta=1.0):
    """Seeded effective-model coefficients (reading A14): (Jk, J2, Jp, Js1, Js2, Js3)
    uniform in [-0.5, 0.5], then Jk -> |Jk| and Jp -> |Jp| so the quartic term confines;
    Jp6 = Jt = 0; wells at +-a with a = lam/omega0^2.  Returned as a plain dict."""
    g = gen(config, 1_000_000 + variant, 0)
    Jk, J2, Jp, j1, j2, j3 = g.uniform(-0.5, 0.5, size=6)
    return dict(Jk=abs(Jk), J2=J2, Jp=abs(Jp), Jp6=0.0, a=lam / omega0 ** 2,
                Js=(j1, j2, j3), Jt=0.0, delta=delta)


def physical_eff(dtau, omega0, c_kin, delta=0.3):
    """Effective model equal to the symmetric part of the bosonic weight:
    Jk = c_kin/dtau, J2 = dtau omega0^2/2 (reading A14, second variant)."""
    return dict(Jk=c_kin / dtau, J2=dtau * omega0 ** 2 / 2.0, Jp=0.0, Jp6=0.0, a=0.0,
                Js=(0.0, 0.0, 0.0), Jt=0.0, delta=delta)
