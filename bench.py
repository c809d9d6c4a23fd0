"""Benchmark of the fermion-weight hot path on one MI355X.

Workload (the 16x16 configuration): 128 chains of a 16x16 periodic lattice (N = 256),
beta = 16 (Ltau = 160, dtau = 0.1), stabilization every n_s = 8 slices, lam = 1.5,
omega0 = 1, Gaussian N(0, 1) phonon fields (seeded), and a seeded symmetric effective
model (on-site x^2, time-adjacent and spatial NN/NNN/third-neighbour couplings).

One step = one SLMC cumulative update of every chain, i.e. every step of the hot path:
  copy x -> x'; one checkerboard Metropolis sweep of the effective model on x' (N Ltau
  site updates); log|det(1 + B...B)| and the Green's function G of every proposal (model
  setup, fused slice scaling, segment products, stabilized QR/UDV chain, recombination,
  FP64 residual step); bosonic action, effective energy and the accept/copy of Eq. 6.
value = chains * steps / time  (fermion log-det + G evaluations per second).

The headline run uses the mixed path that meets the 1e-8 relative log-det target (segment
products on the int8 matrix cores with 5-slice splits, everything else FP64); the FP64
path is timed the same way beside it ("mixed vs FP64").  Also printed: the roofline of
the dominant kernel (HIP events around its launches on its own stream), the roofline of
the slice-product kernel in the overlapped run and with every kernel run alone, the
effective-model sweeps alone, and the other workloads: 4x4 Ltau 40 (64 fields), 8x8
Ltau 80 (256 fields in one call, FP64 against FP32 matrix cores and the int8 split),
the 12x12 Ltau 120 proposal step of 64 chains (sweep + FP64 cumulative accept), the
modified Wolff cluster moves on the same shape, G after every time slice with the CDW
estimators on the 16x16 workload, the paper's DQMC comparison updates (local sweep with
Sherman-Morrison updates, block updates) on the 8x8 and 16x16 workloads, the training of
the effective model on DQMC configurations of the paper's L = 6, the uneven packed batch (L = 8..20) and the headline path's error at couplings 1.0 and 2.0.
The cpu_baseline leg times the FP64 CPU oracle on a bounded sample of the 16x16 fields
(one BLAS thread) and runs it over the GPU outputs of the other legs (every field of the
4x4, 8x8 and 16x16 legs, 8 items of each size class of the uneven batch, 8 of the 64
accept chains), which gives each leg's error against it.
"""

import argparse
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

# dense matrix-core peaks of the MI355X, T(FL)OP/s
PEAK = {"f64": 78.6, "f32": 157.3, "bf16": 2500.0, "i8": 5000.0}
DTYPE = {"fp64": "f64", "fp32": "f32", "bf16x3": "bf16", "bf16x6": "bf16", "int8x5": "i8"}
PRODUCTS = {"fp64": 1, "fp32": 1, "bf16x3": 3, "bf16x6": 6, "int8x5": 15}   # per slice product
# HBM bytes per launch of a kernel class at the 16x16 / 128-chain workload, from rocprofv3
# FETCH_SIZE and WRITE_SIZE counters scaled by what they read for a plain 1 GiB copy
# (factors 2.0 and 1.0).  They are not measured by this script: they are read from the
# committed summary named in TRAFFIC_SOURCE and are valid only for the kernel versions it
# was taken on (the bench line carries the source with the figure).
TRAFFIC = {("qr", "int8x5"): 624.7e6, ("seg_chain", "int8x5"): 85.9e6, ("lu", "int8x5"): 642.4e6,
           ("wy_apply", "int8x5"): 179.5e6, ("vupd", "int8x5"): 181.9e6}
TRAFFIC_SOURCE = ("profiles/fermion_step_16x16_ltau160_int8x5_128chains.md (rocprofv3 --pmc "
                  "FETCH_SIZE / WRITE_SIZE of the seg_chain_i8, qr_k, lu_la_k, wy_apply_reg_k and "
                  "vupd_split_k kernels as of commit dc67a85)")


def run(slmc, torch, md, eff, xs, B, prec, args):
    """Warm-up + timed steps of one precision; returns the measurements."""
    dev = torch.device("cuda:0")
    N = md["Lx"] * md["Ly"]
    m = slmc.model_from_dict(md)
    opt = slmc.options(prec, args.residual, args.acc_chunk, serial=args.serial)
    x_cur = torch.tensor(xs, dtype=torch.float64, device=dev)
    x_prop = torch.empty_like(x_cur)
    G = torch.empty((B, N, N), dtype=torch.float64, device=dev)
    logw, _ = slmc.log_weight(m, x_cur, opt)
    eeff = slmc.eff_energy(m, eff, x_cur)
    seed = 20180216

    def step(k):
        x_prop.copy_(x_cur)
        slmc.eff_sweep(m, eff, x_prop, 1, seed, k)
        return slmc.cumulative_accept(m, eff, x_cur, x_prop, logw, eeff, seed, k, opt, G_prop=G)

    for k in range(args.warmup):
        step(k)
    torch.cuda.synchronize()
    ev0, ev1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    ev0.record()
    t0 = time.perf_counter()
    accs = []
    for k in range(args.warmup, args.warmup + args.steps):
        a, _, _ = step(k)
        accs.append(a)
    ev1.record()
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    ms = ev0.elapsed_time(ev1)
    acc_total = int(sum(int(a.sum().item()) for a in accs))
    # the same number of steps again with the library's per-class HIP events on (they add
    # event records between launches, so they stay out of the timed steps above)
    slmc.profile_reset()
    slmc.profile(True)
    for k in range(args.warmup + args.steps, args.warmup + 2 * args.steps):
        step(k)
    torch.cuda.synchronize()
    slmc.profile(False)
    prof = slmc.profile_read()
    return dict(ms=ms, wall=wall, prof=prof, accept=acc_total / (B * args.steps), opt=opt, m=m)


def sweep_rates(slmc, torch, np, chains, n_sweeps=4, reps=5):
    """Checkerboard sweeps of the effective model alone on the 12x12, Ltau = 120 shape
    (seeded coefficients): site updates per second and algorithmic bytes per second (one
    read and one write of the FP64 field per sweep)."""
    from synth import gen, eff_coefficients
    Lx = Ly = 12
    Lt = 120
    m = slmc.model(Lx, Ly, Lt, 10)
    eff = slmc.eff_model(**eff_coefficients(3, 0, 1.5, delta=0.5))
    x = torch.tensor(gen(3, 999).normal(size=(chains, Lt, Lx * Ly)), dtype=torch.float64, device="cuda:0")
    slmc.eff_sweep(m, eff, x, n_sweeps, 7, 0)
    torch.cuda.synchronize()
    ev0, ev1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    ev0.record()
    for r in range(reps):
        slmc.eff_sweep(m, eff, x, n_sweeps, 7, r + 1)
    ev1.record()
    torch.cuda.synchronize()
    t = ev0.elapsed_time(ev1) / 1e3
    sites = chains * Lx * Ly * Lt * n_sweeps * reps
    return {"chains": chains, "sweeps_per_launch": n_sweeps, "updates_per_s": round(sites / t, 1),
            "algorithmic_GB_per_s": round(16.0 * sites / t / 1e9, 2),
            "working_set_MB": round(8.0 * chains * Lx * Ly * Lt / 1e6, 1)}


def uneven_rates(slmc, torch, np, prec, reps=3):
    """The uneven packed batch: 32 fields for each of L = 8, 12, 16, 20 (Ltau = 10 L,
    n_s = 10, lam = 1.5), items interleaved across the four sizes, log-det + G of all 128 in
    one packed call; then each size class alone (32 items, one call).  Evaluations per
    second from HIP events.  Also returns the packed call's outputs (for the oracle check)."""
    from synth import workload_item, workload_models
    dev = torch.device("cuda:0")
    mds = workload_models("W5")
    models = [slmc.model_from_dict(d) for d in mds]
    order = [(7 * k) % 128 for k in range(128)]
    xs, midx = [], []
    for b in order:
        mi, x = workload_item("W5", b)
        xs.append(x)
        midx.append(mi)
    opt = slmc.options(prec, 1 if prec != "fp64" else 0)

    def packed(sel):
        xsel = [xs[j] for j in sel]
        msel = [midx[j] for j in sel]
        x_off = np.cumsum([0] + [a.size for a in xsel[:-1]])
        g_sizes = [(mds[k]["Lx"] * mds[k]["Ly"]) ** 2 for k in msel]
        g_off = np.cumsum([0] + g_sizes[:-1])
        x = torch.tensor(np.concatenate([a.ravel() for a in xsel]), dtype=torch.float64, device=dev)
        G = torch.empty(int(sum(g_sizes)), dtype=torch.float64, device=dev)
        ws = torch.empty(slmc.workspace_bytes(models, len(sel), opt, model_idx=msel, x_off=x_off,
                                              g_off=g_off), dtype=torch.uint8, device=dev)
        return lambda: slmc.green(models, x, opt, model_idx=msel, x_off=x_off, g_off=g_off,
                                  n_items=len(sel), G=G, ws=ws), g_off

    tuned = {}
    for mi, d in enumerate(mds):
        sel = [j for j in range(128) if midx[j] == mi]
        xc = torch.tensor(np.stack([xs[j] for j in sel]), dtype=torch.float64, device=dev)
        ch, _, rej = slmc.autotune(models[mi], xc, opt)
        tuned["L%d" % d["Lx"]] = dict(ch, rejected=rej)
    fn, g_off = packed(list(range(128)))
    t_all = _timed(torch, fn, reps)
    out = {"packed_128": {"evals_per_s": round(128 / t_all, 1), "ms_per_call": round(t_all * 1e3, 3)}}
    for mi, d in enumerate(mds):
        sel = [j for j in range(128) if midx[j] == mi]
        fc, _ = packed(sel)
        tc = _timed(torch, fc, reps)
        out["L%d_Ltau%d" % (d["Lx"], d["Ltau"])] = {"items": len(sel), "evals_per_s": round(len(sel) / tc, 1),
                                                     "ms_per_call": round(tc * 1e3, 3)}
    out["sum_of_classes_ms"] = round(sum(v["ms_per_call"] for k, v in out.items() if k.startswith("L")), 3)
    out["autotune"] = tuned
    ld, sg, Gp, st = fn()
    torch.cuda.synchronize()
    ld, sg, Gh, st = ld.cpu().numpy(), sg.cpu().numpy(), Gp.cpu().numpy(), st.cpu().numpy()
    checks = []
    for j in range(128):
        d = mds[midx[j]]
        N = d["Lx"] * d["Ly"]
        checks.append(("L%d_Ltau%d" % (d["Lx"], d["Ltau"]), d, xs[j], float(ld[j]), int(st[j]),
                       Gh[g_off[j]:g_off[j] + N * N].reshape(N, N), int(sg[j])))
    return out, checks


def _timed(torch, fn, reps):
    """Seconds per call of fn from HIP events (one untimed call first): the median over
    reps calls, each between its own pair of events, so that a stall of the host between
    two launches of one call does not stand for the call's time."""
    evs = [(torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)) for _ in range(reps)]
    fn()
    torch.cuda.synchronize()
    for e0, e1 in evs:
        e0.record()
        fn()
        e1.record()
    torch.cuda.synchronize()
    ts = sorted(e0.elapsed_time(e1) / 1e3 for e0, e1 in evs)
    return ts[len(ts) // 2]


def _green_all(slmc, torch, np, md, xs, prec, resid, chunk=0, reps=10):
    """log-det + G of all fields in one call: seconds per call and the outputs."""
    m = slmc.model_from_dict(md)
    x = torch.tensor(np.stack(xs), dtype=torch.float64, device="cuda:0")
    opt = slmc.options(prec, resid, chunk)
    t = _timed(torch, lambda: slmc.green(m, x, opt), reps)
    ld, sg, G, st = slmc.green(m, x, opt)
    torch.cuda.synchronize()
    return t, (ld.cpu().numpy(), sg.cpu().numpy(), G.cpu().numpy(), st.cpu().numpy())


def small_rates(slmc, torch, np, reps=20):
    """The small workload (4x4, Ltau = 40, n_s = 10, lam = 1.5, its 64 fields: 48 Gaussian
    and 16 staggered): log-det + G of all 64 in one call, per precision, from HIP events
    over reps calls (latency-bound: a handful of small launches per call)."""
    from synth import workload_item, workload_models
    md = workload_models("W1")[0]
    xs = [workload_item("W1", b)[1] for b in range(64)]
    out, checks = {}, []
    for prec in ("fp64", "int8x5"):
        t, res = _green_all(slmc, torch, np, md, xs, prec, 1 if prec != "fp64" else 0, reps=reps)
        out[prec] = {"evals_per_s": round(64 / t, 1), "ms_per_call": round(t * 1e3, 4)}
        checks += [(prec, md, xs[b], float(res[0][b]), int(res[3][b]), res[2][b], int(res[1][b]))
                   for b in range(64)]
    return out, checks


def fields_8x8_rates(slmc, torch, np, reps=10):
    """8x8 (N = 64), Ltau = 80, n_s = 10, lam = 1.5: 256 seeded Gaussian fields in one
    call, log-det + G: the FP64 path against FP32 matrix-core segment products (FP64
    promotion every k-step of 4, compensation of E's rounding, one residual step) and
    against the int8-slice path, FP64 QR/UDV in all three."""
    from synth import workload_item, workload_models
    md = workload_models("W2")[0]
    xs = [workload_item("W2", b)[1] for b in range(256)]
    out, checks = {}, []
    for prec, resid, chunk in (("fp64", 0, 0), ("fp32", 1, 1), ("int8x5", 1, 0)):
        t, res = _green_all(slmc, torch, np, md, xs, prec, resid, chunk, reps=reps)
        out[prec] = {"evals_per_s": round(256 / t, 1), "ms_per_call": round(t * 1e3, 4)}
        checks += [(prec, md, xs[b], float(res[0][b]), int(res[3][b]), res[2][b], int(res[1][b]))
                   for b in range(256)]
    out["fp32_over_fp64"] = round(out["fp32"]["evals_per_s"] / out["fp64"]["evals_per_s"], 4)
    out["int8x5_over_fp64"] = round(out["int8x5"]["evals_per_s"] / out["fp64"]["evals_per_s"], 4)
    return out, checks


def errors_16x16(slmc, torch, np, prec, lam_idx):
    """GPU outputs of the headline path on all 128 fields of the 16x16 workload at one
    coupling (for the oracle check)."""
    from synth import workload_item, workload_models
    md = workload_models("W4", lam_idx)[0]
    xs = [workload_item("W4", b, lam_idx)[1] for b in range(128)]
    _, res = _green_all(slmc, torch, np, md, xs, prec, 1, reps=1)
    return [(prec, md, xs[b], float(res[0][b]), int(res[3][b]), res[2][b], int(res[1][b]))
            for b in range(128)]


def wolff_12x12(slmc, torch, np, chains=64, n_clusters=4, reps=5):
    """Modified Wolff cluster moves (SM Sec. IV) alone on the 12x12, Ltau = 120 shape with
    the seeded effective model: cluster moves per second, mean cluster size, and the
    whole cumulative proposal (one sweep + the cluster moves in the coin's order); the
    first launch's inputs and outputs for the oracle check."""
    from synth import gen, eff_coefficients, workload_models
    md = workload_models("W3")[0]
    m = slmc.model_from_dict(md)
    effd = eff_coefficients(3, 0, md["lam"], delta=0.5)
    eff = slmc.eff_model(**effd)
    x0 = gen(3, 501).normal(size=(chains, md["Ltau"], md["Lx"] * md["Ly"]))
    x = torch.tensor(x0, dtype=torch.float64, device="cuda:0")
    seed = 1802061771
    sizes0 = slmc.eff_wolff(m, eff, x, n_clusters, seed, 0)
    torch.cuda.synchronize()
    first = dict(md=md, eff=effd, seed=seed, n_clusters=n_clusters, x_in=x0, x_out=x.cpu().numpy(),
                 sizes=sizes0.cpu().numpy())
    k = [0]

    def clusters():
        k[0] += 1
        slmc.eff_wolff(m, eff, x, n_clusters, seed, k[0])

    def proposal():
        k[0] += 1
        slmc.eff_propose(m, eff, x, 1, n_clusters, seed, k[0])

    t_w = _timed(torch, clusters, reps)
    t_p = _timed(torch, proposal, reps)
    sz = slmc.eff_wolff(m, eff, x, n_clusters, seed, 10 ** 6).float().mean().item()
    out = {"chains": chains, "clusters_per_launch": n_clusters,
           "cluster_moves_per_s": round(chains * n_clusters / t_w, 1),
           "ms_per_launch": round(t_w * 1e3, 4), "mean_cluster_size": round(sz, 2),
           "sites": md["Lx"] * md["Ly"],
           "proposal_ms": round(t_p * 1e3, 4),
           "proposals_per_s": round(chains / t_p, 1)}
    return out, first


def slices_16x16(slmc, torch, np, items=32, reps=2):
    """G after every time slice (SM Eq. S3) and the CDW estimators on the 16x16, Ltau = 160
    workload (FP64 evaluations every n_wrap slices, FP64 propagation between): slices per
    second at n_wrap = 8 and 40, and the n_wrap = 8 outputs of two fields on sampled slices
    for the oracle check."""
    from synth import workload_item, workload_models
    md = workload_models("W4", 1)[0]
    m = slmc.model_from_dict(md)
    xs = [workload_item("W4", b, 1)[1] for b in range(items)]
    x = torch.tensor(np.stack(xs), dtype=torch.float64, device="cuda:0")
    opt = slmc.options("fp64")
    out = {"items": items, "Ltau": md["Ltau"]}
    for nw in (8, 40):
        t = _timed(torch, lambda: slmc.green_slices(m, x, nw, opt), reps)
        out["n_wrap_%d" % nw] = {"ms_per_call": round(t * 1e3, 3),
                                 "slices_per_s": round(items * md["Ltau"] / t, 1),
                                 "evaluations_per_call": items * ((md["Ltau"] + nw - 1) // nw)}
    s_nn, m_st, st, G = slmc.green_slices(m, x[:2].contiguous(), 8, opt, want_g=True)
    sl = [0, 3, 6, 7, 100, 159]
    first = dict(md=md, x=[xs[0], xs[1]], slices=sl, G=G.cpu().numpy()[:, sl], s_nn=s_nn.cpu().numpy()[:, sl],
                 m_st=m_st.cpu().numpy()[:, sl], status=st.cpu().numpy())
    out["cdw_s_nn_mean"] = round(float(s_nn.mean().item()), 6)
    return out, first


def dqmc_rates(slmc, torch, np, wl, chains, n_rec, reps=1):
    """The paper's comparison method on the GPU (SM Sec. I): one DQMC local sweep of every
    chain (N Ltau sequential local updates per chain, each with its O(N^2) Sherman-Morrison
    update; G re-evaluated every n_rec slices) and 4 column block updates, FP64.  Sweep time,
    site updates per second and acceptance, from HIP events."""
    from synth import workload_item, workload_models
    md = workload_models(wl, 1 if wl == "W4" else 0)[0]
    m = slmc.model_from_dict(md)
    N, Lt = md["Lx"] * md["Ly"], md["Ltau"]
    xs = [workload_item(wl, b % 128, 1 if wl == "W4" else 0)[1] for b in range(chains)]
    x = torch.tensor(np.stack(xs), dtype=torch.float64, device="cuda:0")
    opt = slmc.options("fp64")
    k = [0]
    accs = []

    def sweep():
        k[0] += 1
        a, _, _ = slmc.dqmc_sweep(m, x, 0.8, n_rec, 2018, k[0], opt)
        accs.append(a)

    t = _timed(torch, sweep, reps)
    acc = float(torch.stack(accs[-reps:]).double().mean().item()) / (N * Lt)
    logw, _ = slmc.log_weight(m, x, opt)

    def block():
        k[0] += 1
        slmc.dqmc_block(m, x, logw, 4, 2018, k[0], opt)

    tb = _timed(torch, block, reps)
    return {"chains": chains, "N": N, "Ltau": Lt, "n_rec": n_rec, "sweep_ms": round(t * 1e3, 3),
            "site_updates_per_s": round(chains * N * Lt / t, 1), "local_accept_rate": round(acc, 4),
            "block_updates": 4, "block_ms": round(tb * 1e3, 3)}


def train_6x6(slmc, torch, np, chains=64, burn=8, keep=16):
    """Training the effective model on the paper's L = 6 (Eq. 5, SM Sec. III; beta = 4,
    Ltau = 40, g = 1, Omega = 0.5, i.e. the paper's lambda = 0.5): DQMC local sweeps of 64
    chains generate the configurations (burn-in, then one per chain per sweep), their log
    weights, and the least-squares fit of the paper's five terms; wall time of each part
    from HIP events, and the data for the oracle check."""
    from synth import gen
    md = dict(Lx=6, Ly=6, Ltau=40, n_s=10, t=1.0, mu=0.0, dtau=0.1, lam=1.0, omega0=0.5, c_kin=0.5)
    m = slmc.model_from_dict(md)
    x = torch.tensor(gen(6, 0).normal(size=(chains, 40, 36)), dtype=torch.float64, device="cuda:0")
    ev = [torch.cuda.Event(enable_timing=True) for _ in range(4)]
    confs = []
    ev[0].record()
    for sw in range(burn + keep):
        slmc.dqmc_sweep(m, x, 1.0, 10, 1802, sw)
        if sw >= burn:
            confs.append(x.clone())
    ev[1].record()
    X = torch.cat(confs)
    lw, st = slmc.log_weight(m, X)
    ev[2].record()
    terms = ("Jk", "Jp", "Jp6", "Js0", "Jt")
    coef, F = slmc.eff_fit(m, X, lw, terms=terms)
    ev[3].record()
    torch.cuda.synchronize()
    c = coef.cpu().numpy()
    Fh, lwh = F.cpu().numpy(), lw.cpu().numpy()
    mask = np.array([t in terms for t in slmc.TERMS], dtype=float)
    pred = c[0] - Fh @ (c[1:] * mask)
    r2 = 1.0 - float(np.sum((lwh - pred) ** 2) / np.sum((lwh - lwh.mean()) ** 2))
    out = {"configurations": int(X.shape[0]), "sweeps": burn + keep, "chains": chains,
           "dqmc_ms": round(ev[0].elapsed_time(ev[1]), 2), "log_weight_ms": round(ev[1].elapsed_time(ev[2]), 3),
           "fit_ms": round(ev[2].elapsed_time(ev[3]), 3), "status_ok": bool(torch.all(st == 0).item()),
           "E0": float(c[0]), "J": {t: float(c[1 + k]) for k, t in enumerate(slmc.TERMS) if t in terms},
           "r2": round(r2, 6)}
    first = dict(md=md, X=X.cpu().numpy(), logw=lwh, F=Fh, coef=c, terms=terms)
    return out, first


def accept_12x12(slmc, torch, np, steps=10):
    """64 chains of the 12x12, Ltau = 120 shape (n_s = 10, lam = 1.5) with the seeded
    effective model (couplings out to the third neighbour): one proposal = copy, one
    checkerboard sweep (N Ltau site updates), FP64 cumulative accept (log-det of every
    proposal, bosonic action, effective energy, Eq. 6).  Proposals per second of the whole
    step and of the accept call alone (HIP events), and the first proposal's inputs and
    outputs for the oracle check."""
    from synth import gen, eff_coefficients, workload_models
    md = workload_models("W3")[0]
    m = slmc.model_from_dict(md)
    effd = eff_coefficients(3, 0, md["lam"], delta=0.5)
    eff = slmc.eff_model(**effd)
    chains = 64
    x0 = gen(3, 500).normal(size=(chains, md["Ltau"], md["Lx"] * md["Ly"]))
    x_cur = torch.tensor(x0, dtype=torch.float64, device="cuda:0")
    x_prop = torch.empty_like(x_cur)
    opt = slmc.options("fp64")
    logw, _ = slmc.log_weight(m, x_cur, opt)
    eeff = slmc.eff_energy(m, eff, x_cur)
    seed = 1802061770
    logw0, eeff0 = logw.cpu().numpy(), eeff.cpu().numpy()
    x_prop.copy_(x_cur)
    slmc.eff_sweep(m, eff, x_prop, 1, seed, 0)
    xp0 = x_prop.cpu().numpy()
    acc0, lr0, st0 = slmc.cumulative_accept(m, eff, x_cur, x_prop, logw, eeff, seed, 0, opt)
    first = dict(md=md, eff=effd, seed=seed, x_cur=x0, x_prop=xp0, logw=logw0, eeff=eeff0,
                 accepted=acc0.cpu().numpy(), log_ratio=lr0.cpu().numpy(), status=st0.cpu().numpy())
    ev = [torch.cuda.Event(enable_timing=True) for _ in range(2 * steps + 2)]
    torch.cuda.synchronize()
    ev[0].record()
    for k in range(1, steps + 1):
        x_prop.copy_(x_cur)
        slmc.eff_sweep(m, eff, x_prop, 1, seed, k)
        ev[2 * k].record()
        slmc.cumulative_accept(m, eff, x_cur, x_prop, logw, eeff, seed, k, opt)
        ev[2 * k + 1].record()
    torch.cuda.synchronize()
    total = ev[0].elapsed_time(ev[2 * steps + 1]) / 1e3
    acc_t = sum(ev[2 * k].elapsed_time(ev[2 * k + 1]) for k in range(1, steps + 1)) / 1e3
    out = {"chains": chains, "steps": steps,
           "proposals_per_s": round(chains * steps / total, 1),
           "accept_only_proposals_per_s": round(chains * steps / acc_t, 1),
           "ms_per_step": round(total * 1e3 / steps, 4),
           "accept_ms_per_step": round(acc_t * 1e3 / steps, 4)}
    return out, first


def roofline(prof, prec, md, B, steps, counters_apply, kernel=None):
    """A kernel class (default: the dominant one, largest event time in the timed region)
    against its peak: achieved = algorithmic work per launch / average launch time."""
    N, Lt, n_s = md["Lx"] * md["Ly"], md["Ltau"], md["n_s"]
    nseg = (Lt + n_s - 1) // n_s
    dom = kernel or max(prof, key=lambda k: prof[k][0])
    dom_ms, dom_n = prof[dom]
    # per-evaluation algorithmic flops of each class (FP64-equivalent)
    per_eval = {
        "seg_chain": 2.0 * N ** 3 * (Lt - nseg),   # n_s - 1 products per segment
        "qr": (4.0 / 3.0) * N ** 3 * nseg,         # Householder QR of N x N per block
        "wy_apply": 2.0 * N ** 3 * nseg,           # S_k Q_{k-1}
        "vupd": 1.0 * N ** 3 * nseg,               # triangular times dense
        "lu": (2.0 / 3.0) * N ** 3,
        "lu_solve": 4.0 * N ** 3,                  # solve + refinement solve
        "residual": 2.0 * N ** 3,
        "eff_sweep": 0.0,
    }
    launches_per_step = dom_n / steps if dom_n else 1.0
    work_per_launch = per_eval.get(dom, 0.0) * B / launches_per_step
    t_launch = dom_ms / dom_n / 1e3 if dom_n else float("nan")
    dtype = DTYPE[prec] if dom == "seg_chain" else "f64"
    ops = work_per_launch * (PRODUCTS[prec] if dom == "seg_chain" else 1)
    achieved = ops / t_launch / 1e12 if dom_n else 0.0
    return {"kernel": dom, "bound": "mfma", "achieved": round(achieved, 3), "peak": PEAK[dtype],
            "unit": "TOP/s" if dtype == "i8" else "TFLOP/s", "frac": round(achieved / PEAK[dtype], 4),
            "traffic": TRAFFIC.get((dom, prec)) if counters_apply else None,
            "traffic_source": TRAFFIC_SOURCE if counters_apply and (dom, prec) in TRAFFIC else None,
            "avg_launch_ms": round(t_launch * 1e3, 4),
            "work_per_launch": ops,
            "fp64_equiv_tflops": round(work_per_launch / t_launch / 1e12, 3) if dom_n else None,
            "per_class_ms_per_step": {k: round(v[0] / steps, 3) for k, v in prof.items() if v[1]}}


def path_roofline(prec, md, value):
    """Whole evaluation against the matrix-core peaks: T_roof = F_lo / P_lo + F_hi / P_64 per
    evaluation, with F_lo the segment products (2 N^3 (n_s - 1) per block, times the number of
    split products, in the precision of the path) and F_hi the FP64 rest (S U, Householder QR
    with Q and R P^T V: (2 + 11/3) N^3 per block; LU and N-column solve (8/3) N^3; residual
    step 8 N^3 when the path runs it)."""
    N, Lt, n_s = md["Lx"] * md["Ly"], md["Ltau"], md["n_s"]
    m = (Lt + n_s - 1) // n_s
    n3 = float(N) ** 3
    seg = 2.0 * n3 * (Lt - m)
    f_hi = (2.0 + 11.0 / 3.0) * n3 * m + (8.0 / 3.0) * n3 + (8.0 * n3 if prec != "fp64" else 0.0)
    if prec == "fp64":
        t = (seg + f_hi) / (PEAK["f64"] * 1e12)
    else:
        t = seg * PRODUCTS[prec] / (PEAK[DTYPE[prec]] * 1e12) + f_hi / (PEAK["f64"] * 1e12)
    return {"t_roof_us_per_eval": round(t * 1e6, 2), "ceiling_evals_per_s": round(1.0 / t, 1),
            "frac": round(value * t, 4)}


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=10)
    ap.add_argument("--warmup", type=int, default=2)
    ap.add_argument("--precision", default="int8x5", choices=sorted(DTYPE))
    ap.add_argument("--acc-chunk", type=int, default=0)
    ap.add_argument("--residual", type=int, default=1)
    ap.add_argument("--chains", type=int, default=128)
    ap.add_argument("--lam", type=float, default=1.5)
    ap.add_argument("--serial", action="store_true",
                    help="keep the segment products on the caller's stream (no overlap)")
    ap.add_argument("--no-fp64", action="store_true", help="skip the FP64 comparison run")
    ap.add_argument("--no-alone", action="store_true",
                    help="skip the serial-schedule run of the slice-product kernel")
    ap.add_argument("--cpu-sample", type=int, default=128,
                    help="oracle items for cpu_baseline, about 10-30 s of CPU work (0: skip)")
    ap.add_argument("--cpu-all-threads", action="store_true",
                    help="also time the oracle with the BLAS library's default thread count "
                         "(slower than one thread at these sizes)")
    ap.add_argument("--no-tune", action="store_true",
                    help="keep the default schedule and tile choices (no autotuning)")
    ap.add_argument("--no-workloads", action="store_true",
                    help="skip the legs of the other workloads (4x4, 8x8, 12x12 accept, uneven "
                         "packed batch, 16x16 error by coupling), e.g. for profiling runs")
    ap.add_argument("--copy-calibration", type=int, default=0, metavar="MIB",
                    help="only run a plain device-to-device copy of MIB mebibytes (reference "
                         "for the HBM byte counters) and exit")
    args = ap.parse_args()
    if args.gpus != 1:
        print("bench.py measures one GPU only: this build runs the hot path on a single MI355X "
              "(chains shard across GPUs with no exchange; no multi-GPU run is part of it).",
              file=sys.stderr)
        sys.exit(2)

    import numpy as np
    import torch

    if args.copy_calibration > 0:
        n = args.copy_calibration * (1 << 20) // 8
        src = torch.ones(n, dtype=torch.float64, device="cuda:0")
        dst = torch.empty_like(src)
        torch.cuda.synchronize()
        dst.copy_(src)
        torch.cuda.synchronize()
        print(json.dumps({"copy_calibration_bytes_read": 8 * n, "copy_calibration_bytes_written": 8 * n}))
        return

    import paper_1802_06177_amd as slmc
    from synth import workload_item, workload_models, eff_coefficients

    lam_idx = {1.0: 0, 1.5: 1, 2.0: 2}.get(args.lam, 1)
    md = dict(workload_models("W4", lam_idx)[0])
    md["lam"] = args.lam
    B = args.chains
    eff = slmc.eff_model(**eff_coefficients(4, 0, args.lam, delta=0.6))
    xs = np.stack([workload_item("W4", b % 128, lam_idx)[1] for b in range(B)])

    # the autotuner picks the schedule and tile choices of both paths on these fields first
    tune = {}
    for p in ([args.precision] + ([] if args.precision == "fp64" or args.no_fp64 else ["fp64"])):
        o = slmc.options(p, args.residual if p != "fp64" else 0, args.acc_chunk)
        if not args.no_tune and not args.serial:
            ch, tried, rej = slmc.autotune(slmc.model_from_dict(md),
                                           torch.tensor(xs, dtype=torch.float64, device="cuda:0"), o)
            tune[p] = dict(ch, source="tuned in this run", candidates=tried, rejected=rej)
        else:
            ch, tuned = slmc.tuning(slmc.model_from_dict(md), B, o)
            tune[p] = dict(ch, source="cache file" if tuned else "defaults")
    _progress("schedule and tile choices: %s" % tune)
    main_run = run(slmc, torch, md, eff, xs, B, args.precision, args)
    _progress("headline run done: %.1f evals/s" % (B * args.steps / (main_run["ms"] / 1e3)))
    ms_per_step = main_run["ms"] / args.steps
    value = B * args.steps / (main_run["ms"] / 1e3)
    roof = roofline(main_run["prof"], args.precision, md, B, args.steps,
                    counters_apply=(B == 128 and args.lam == 1.5))

    # the slice-product kernel on its own: its event times in the overlapped run include the
    # time it shares the compute units with the QR chain, so it is also timed with the
    # serial schedule (every kernel alone on the caller's stream)
    seg_rate = None
    if "seg_chain" in main_run["prof"]:
        keep = ("kernel", "bound", "achieved", "peak", "unit", "frac", "avg_launch_ms")
        r_over = roofline(main_run["prof"], args.precision, md, B, args.steps, False, "seg_chain")
        seg_rate = {"schedule_" + ("serial" if args.serial else "overlapped"): {k: r_over[k] for k in keep}}
        if not args.serial and not args.no_alone:
            args_alone = argparse.Namespace(**vars(args))
            args_alone.serial = True
            r_al = run(slmc, torch, md, eff, xs, B, args.precision, args_alone)
            r_alone = roofline(r_al["prof"], args.precision, md, B, args.steps, False, "seg_chain")
            seg_rate["schedule_serial"] = {k: r_alone[k] for k in keep}
            _progress("serial-schedule run done")

    fp64 = None
    if args.precision != "fp64" and not args.no_fp64:
        r64 = run(slmc, torch, md, eff, xs, B, "fp64", args)
        v64 = B * args.steps / (r64["ms"] / 1e3)
        fp64 = {"value": round(v64, 3),
                "ms_per_step": round(r64["ms"] / args.steps, 4),
                "mixed_over_fp64": round(r64["ms"] / main_run["ms"], 4),
                "path_roofline": path_roofline("fp64", md, v64)}
        _progress("FP64 run done: %.1f evals/s" % v64)

    # the effective-model sweep alone on the 12x12 shape: 64 chains (L2-resident) and 2048
    # chains (a working set above the 256 MB last-level cache)
    sweep = {"12x12x120_64": sweep_rates(slmc, torch, np, 64),
             "12x12x120_2048": sweep_rates(slmc, torch, np, 2048, n_sweeps=1, reps=3)}
    _progress("sweep legs done")

    # the other workloads, timed on the GPU; their outputs are checked against the oracle in
    # the cpu_baseline leg below
    legs, checks = {}, {}
    if not args.no_workloads:
        legs["small_4x4"], checks["small_4x4"] = small_rates(slmc, torch, np)
        _progress("4x4 leg done")
        legs["fields_8x8_ltau80"], checks["fields_8x8_ltau80"] = fields_8x8_rates(slmc, torch, np)
        _progress("8x8 leg done")
        legs["accept_12x12_ltau120"], checks["accept_12x12_ltau120"] = accept_12x12(slmc, torch, np)
        _progress("12x12 accept leg done")
        legs["wolff_12x12_ltau120"], checks["wolff_12x12_ltau120"] = wolff_12x12(slmc, torch, np)
        _progress("12x12 Wolff leg done")
        legs["slices_16x16_ltau160"], checks["slices_16x16_ltau160"] = slices_16x16(slmc, torch, np)
        _progress("16x16 G-slices leg done")
        legs["dqmc"] = {"8x8_ltau80": dqmc_rates(slmc, torch, np, "W2", 64, 10),
                        "16x16_ltau160": dqmc_rates(slmc, torch, np, "W4", B, 8)}
        _progress("DQMC comparison leg done")
        legs["train_6x6_ltau40"], checks["train_6x6_ltau40"] = train_6x6(slmc, torch, np)
        _progress("training leg done")
        legs["uneven_packed"] = {}
        checks["uneven_packed"] = []
        for prec in (args.precision, "fp64"):
            legs["uneven_packed"][prec], ch = uneven_rates(slmc, torch, np, prec)
            seen = {}
            for c in ch:     # the first 8 items of each size class
                seen[c[0]] = seen.get(c[0], 0) + 1
                if seen[c[0]] <= 8:
                    checks["uneven_packed"].append((prec + ":" + c[0],) + c[1:])
            _progress("uneven leg (%s) done" % prec)
        checks["errors_16x16_by_lam"] = []
        for li in (0, 2):
            checks["errors_16x16_by_lam"] += errors_16x16(slmc, torch, np, args.precision, li)
        _progress("16x16 error leg done")

    # CPU oracle: timed on one BLAS thread on a bounded sample of the 16x16 fields (the
    # baseline), and run over the outputs of the GPU legs above (uneven batch and accept
    # step sampled), which gives the error of each leg against it
    cpu = None
    err = None
    if args.cpu_sample > 0:
        import oracle
        E = oracle.expk(oracle.hopping_matrix(md["Lx"], md["Ly"], md["t"], md["mu"]), md["dtau"])
        ns = min(args.cpu_sample, B)
        xsamp = xs[:ns]
        ld_g, sg_g, G_g, st_g = slmc.green(main_run["m"], torch.tensor(xsamp, device="cuda:0"), main_run["opt"])
        torch.cuda.synchronize()
        ld_g, sg_g, G_g, st_g = ld_g.cpu().numpy(), sg_g.cpu().numpy(), G_g.cpu().numpy(), st_g.cpu().numpy()

        def oracle_rate(items):
            t1 = time.perf_counter()
            out = [oracle.logdet_green(E, xsamp[k], md["dtau"], md["lam"], md["n_s"]) for k in items]
            return out, len(items) / (time.perf_counter() - t1)

        what = ("of the %d fields (16x16, Ltau=160, n_s=8, lam=%.1f), log-det + G, numpy/scipy FP64 "
                "(LAPACK QRP + LU)" % (B, md["lam"]))
        host = _host_info()
        from threadpoolctl import threadpool_info, threadpool_limits
        threads = max([d.get("num_threads", 1) for d in threadpool_info()] + [1])
        # one thread is the faster setting for these 256 x 256 factorizations (the BLAS
        # threads cost more than they bring), so it is the baseline; the library's default
        # thread count is timed beside it on a few fields
        with threadpool_limits(limits=1):
            refs, r1 = oracle_rate(range(ns))
        _progress("oracle baseline (one thread, %d fields) done" % ns)
        cpu = {"value": round(r1, 4), "unit": "evals/s", "cores": 1, "kind": "oracle",
               "sample": "%d %s, one BLAS thread" % (ns, what),
               "cpu_model": host["cpu_model"], "host_cpus": host["cpus"],
               "blas_threads_default": int(threads)}
        if args.cpu_all_threads:
            _, rall = oracle_rate(range(min(6, ns)))
            cpu["all_threads"] = {"value": round(rall, 4), "cores": int(threads),
                                  "sample": "%d of the same fields" % min(6, ns)}
            _progress("oracle on %d BLAS threads done" % threads)
        err = {"max_rel_logdet": float(max(abs(ld_g[k] - refs[k][0]) / abs(refs[k][0]) for k in range(ns))),
               "max_per_site_logdet": float(max(abs(ld_g[k] - refs[k][0]) for k in range(ns)) / (md["Lx"] * md["Ly"])),
               "max_abs_G": float(max(np.max(np.abs(G_g[k] - refs[k][2])) for k in range(ns))),
               "signs_equal": bool(all(int(sg_g[k]) == refs[k][1] for k in range(ns))),
               "status_ok": bool(np.all(st_g == 0)),
               "items": ns, "precision": args.precision, "lam": md["lam"]}
        if checks:
            t1 = time.perf_counter()
            with threadpool_limits(limits=1):
                summary, n_eval = _oracle_checks(checks)
            cpu["workload_checks"] = {"oracle_evaluations": n_eval, "blas_threads": 1,
                                      "wall_s": round(time.perf_counter() - t1, 2)}
            for name, tab in summary.items():
                legs.setdefault(name, {})["error_vs_oracle"] = tab
            err["by_lam"] = legs.pop("errors_16x16_by_lam")["error_vs_oracle"]
            err["by_lam"]["lam=1.5"] = {args.precision: {k: err[k] for k in (
                "max_rel_logdet", "max_per_site_logdet", "max_abs_G", "items")}}

    out = {
        "metric": "fermion logdet+G evals/s at N=256,Ltau=160: mixed vs FP64, <=1e-8 rel err",
        "value": round(value, 3), "unit": "evals/s", "n_gpus": 1, "steps": args.steps,
        "warmup": args.warmup, "ms_per_step": round(ms_per_step, 4), "higher_is_better": True,
        "scaling": "weak", "vs_baseline": None, "dtype": DTYPE[args.precision], "data": "synthetic",
        "config": {"workload": "16x16 (N=256), beta=16 (Ltau=160), n_s=8, lam=%.1f, omega0=1, "
                               "%d chains; step = sweep + logdet+G of proposals + accept" % (md["lam"], B),
                   "precision": args.precision, "acc_chunk": args.acc_chunk,
                   "residual_steps": args.residual, "global_batch": B, "parallelism": "none",
                   "schedule": "serial" if args.serial else "overlapped"},
        "autotune": tune,
        "roofline": roof, "slice_products": seg_rate, "path_roofline": path_roofline(args.precision, md, value),
        "cpu_baseline": cpu, "error_vs_oracle": err,
        "fp64_path": fp64,
        "sweep_only": sweep,
        "accept_rate": round(main_run["accept"], 4), "wall_s": round(main_run["wall"], 3),
    }
    out.update(legs)
    print(json.dumps(out), flush=True)


def _progress(msg):
    print("[bench %.1f s] %s" % (time.perf_counter() - _T0, msg), file=sys.stderr, flush=True)


_T0 = time.perf_counter()


def _host_info():
    model = "unknown"
    try:
        with open("/proc/cpuinfo") as f:
            for line in f:
                if line.startswith("model name"):
                    model = line.split(":", 1)[1].strip()
                    break
    except OSError:
        pass
    try:
        cpus = len(os.sched_getaffinity(0))
    except AttributeError:
        cpus = os.cpu_count() or 1
    return {"cpu_model": model, "cpus": cpus}


_E_CACHE = {}


def oracle_E(d):
    import oracle
    key = (d["Lx"], d["Ly"], d["t"], d["mu"], d["dtau"])
    if key not in _E_CACHE:
        _E_CACHE[key] = oracle.expk(oracle.hopping_matrix(d["Lx"], d["Ly"], d["t"], d["mu"]), d["dtau"])
    return _E_CACHE[key]


def _oracle_fermion(task):
    """One oracle evaluation against one GPU result: (label, rel log-det error, per-site
    error, max |dG|, sign equal, status ok)."""
    import numpy as np
    import oracle
    label, d, x, ld, st, G, sg = task
    key = (d["Lx"], d["Ly"], d["t"], d["mu"], d["dtau"])
    if key not in _E_CACHE:
        _E_CACHE[key] = oracle.expk(oracle.hopping_matrix(d["Lx"], d["Ly"], d["t"], d["mu"]), d["dtau"])
    ref, rs, rG = oracle.logdet_green(_E_CACHE[key], x, d["dtau"], d["lam"], d["n_s"])
    return (label, abs(ld - ref) / abs(ref), abs(ld - ref) / (d["Lx"] * d["Ly"]),
            float(np.max(np.abs(G - rG))), sg == rs, st == 0, d["lam"])


def _oracle_accept(task):
    """The oracle's sweep and cumulative accept of one chain's first proposal against the
    GPU's: (max |x'_gpu - x'_oracle|, decision equal, |log r - log r_oracle|, near-tie)."""
    import numpy as np
    import oracle
    from oracle.effective import EffModel
    from oracle.philox import philox4x32_10, uniform01
    d, effd, seed, c, x_cur, x_prop, logw, eeff, acc, lr = task
    key = (d["Lx"], d["Ly"], d["t"], d["mu"], d["dtau"])
    if key not in _E_CACHE:
        _E_CACHE[key] = oracle.expk(oracle.hopping_matrix(d["Lx"], d["Ly"], d["t"], d["mu"]), d["dtau"])
    E = _E_CACHE[key]
    om = EffModel(**{**effd, "Js": tuple(effd["Js"])})
    xo = x_cur.copy()
    margins = []
    oracle.sweep(xo, d["Lx"], d["Ly"], om, 1, seed, 0, c, margins=margins)
    ld = oracle.logdet_green(E, x_cur, d["dtau"], d["lam"], d["n_s"])[0]
    lw0 = oracle.log_weight(ld, x_cur, d["lam"], d["omega0"], d["dtau"], d["c_kin"])
    e0 = oracle.eff_energy(x_cur, d["Lx"], d["Ly"], om)
    a, log_r, _, _ = oracle.cumulative_accept(E, d["Lx"], d["Ly"], d["dtau"], d["lam"], d["omega0"],
                                              d["c_kin"], d["n_s"], om, x_cur, xo, lw0, e0, seed, 0, c)
    kk = (seed & 0xFFFFFFFF, (seed >> 32) & 0xFFFFFFFF)
    u = float(uniform01(philox4x32_10((0xFFFFFFFF, 0xFFFFFFFF, 0, c), kk)[0]))
    return (float(np.max(np.abs(x_prop - xo))), bool(acc) == a, abs(lr - log_r),
            int(abs(np.log(u) - log_r) <= 1e-8), int(np.sum(np.abs(margins) <= 1e-12)),
            abs(logw - lw0) / abs(lw0), bool(a))


def _oracle_checks(checks):
    """Runs the oracle over the GPU outputs of the workload legs, one evaluation after
    another in this process (progress on stderr every 50)."""
    import numpy as np
    ferm = [(name, t) for name, lst in checks.items()
            if name not in ("accept_12x12_ltau120", "wolff_12x12_ltau120", "slices_16x16_ltau160",
                            "train_6x6_ltau40")
            for t in lst]
    acc = checks.get("accept_12x12_ltau120")
    acc_tasks = []
    if acc:
        for c in range(min(8, len(acc["accepted"]))):
            acc_tasks.append((acc["md"], acc["eff"], acc["seed"], c, acc["x_cur"][c], acc["x_prop"][c],
                              float(acc["logw"][c]), float(acc["eeff"][c]), int(acc["accepted"][c]),
                              float(acc["log_ratio"][c])))
    order = list(range(len(ferm)))
    ff, fa = [], []
    for j, k in enumerate(order):
        ff.append(_oracle_fermion(ferm[k][1]))
        if (j + 1) % 50 == 0:
            _progress("oracle checks: %d of %d evaluations" % (j + 1, len(order)))
    for t in acc_tasks:
        fa.append(_oracle_accept(t))
    wf = checks.get("wolff_12x12_ltau120")
    wres = None
    if wf:
        from oracle.effective import EffModel
        from oracle.wolff import wolff as o_wolff
        d = wf["md"]
        om = EffModel(**{**wf["eff"], "Js": tuple(wf["eff"]["Js"])})
        same, ties, n = 0, 0, min(4, len(wf["sizes"]))
        for c in range(n):
            xo = wf["x_in"][c].copy()
            margins = []
            so = o_wolff(xo, d["Lx"], d["Ly"], om, wf["n_clusters"], wf["seed"], 0, c, margins=margins)
            ties += int(np.sum(np.abs(np.asarray(margins)) <= 1e-12))
            same += int(list(wf["sizes"][c]) == so and np.array_equal(wf["x_out"][c], xo))
        wres = {"chains": n, "fields_and_clusters_equal": same, "bond_near_ties": ties}
    _progress("oracle checks done: %d + %d evaluations" % (len(ff), len(fa)))
    summary = {}
    for k, r in zip(order, ff):
        name = ferm[k][0]
        label, rel, site, dg, sg_ok, st_ok, lam = r
        sub = summary.setdefault(name, {})
        if name == "errors_16x16_by_lam":
            sub = sub.setdefault("lam=%.1f" % lam, {})
        t = sub.setdefault(label, {"max_rel_logdet": 0.0, "max_per_site_logdet": 0.0, "max_abs_G": 0.0,
                                   "items": 0, "signs_equal": True, "status_ok": True})
        t["max_rel_logdet"] = max(t["max_rel_logdet"], rel)
        t["max_per_site_logdet"] = max(t["max_per_site_logdet"], site)
        t["max_abs_G"] = max(t["max_abs_G"], dg)
        t["items"] += 1
        t["signs_equal"] &= bool(sg_ok)
        t["status_ok"] &= bool(st_ok)
    if fa:
        a = np.array([[r[0], r[1], r[2], r[3], r[4], r[5], r[6]] for r in fa], dtype=float)
        summary["accept_12x12_ltau120"] = {
            "chains": len(fa), "max_abs_dx_after_sweep": float(a[:, 0].max()),
            "decisions_equal": int(a[:, 1].sum()), "accepted_by_oracle": int(a[:, 6].sum()),
            "max_abs_dlog_r": float(a[:, 2].max()), "accept_near_ties": int(a[:, 3].sum()),
            "sweep_near_ties": int(a[:, 4].sum()), "max_rel_logw_current": float(a[:, 5].max())}
    if wres:
        summary["wolff_12x12_ltau120"] = wres
    sc = checks.get("slices_16x16_ltau160")
    if sc:
        d = sc["md"]
        E = oracle_E(d)
        from oracle.measure import green_slices, cdw_estimators
        dg, ds = 0.0, 0.0
        for b, xb in enumerate(sc["x"]):
            ref = green_slices(E, xb, d["dtau"], d["lam"], d["n_s"], slices=sc["slices"])
            for k in range(len(sc["slices"])):
                dg = max(dg, float(np.max(np.abs(sc["G"][b, k] - ref[k]))))
                ds = max(ds, abs(sc["s_nn"][b, k] - cdw_estimators(ref[k], d["Lx"], d["Ly"])[0]))
        summary["slices_16x16_ltau160"] = {"fields": len(sc["x"]), "slices": sc["slices"], "n_wrap": 8,
                                           "max_abs_G": dg, "max_abs_s_nn": ds,
                                           "status_ok": bool(np.all(sc["status"] == 0))}
    tc = checks.get("train_6x6_ltau40")
    if tc:
        from oracle.train import features as o_features, fit as o_fit, TERMS
        d = tc["md"]
        a = d["lam"] / d["omega0"] ** 2
        Fo = np.array([o_features(xc, d["Lx"], d["Ly"], a) for xc in tc["X"]])
        mask = [int(t in tc["terms"]) for t in TERMS]
        E0, J = o_fit(Fo, tc["logw"], mask)
        ref = np.concatenate([[E0], J])
        summary["train_6x6_ltau40"] = {
            "configurations": int(len(Fo)),
            "max_rel_features": float(np.max(np.abs(tc["F"] - Fo) / np.maximum(1.0, np.abs(Fo)))),
            "max_rel_coef": float(np.max(np.abs(tc["coef"] - ref)) / np.max(np.abs(ref)))}
    return summary, len(ferm) + len(acc_tasks) + (wres["chains"] if wres else 0) + \
        (2 * len(sc["slices"]) if sc else 0)


if __name__ == "__main__":
    main()
