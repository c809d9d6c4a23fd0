"""GPU parity of the fermion weight (SM Eqs. S2, S3): the HIP path through the C ABI
against the FP64 CPU oracle on the same seeded inputs.

Bars (max over items): FP64 path: relative log-det error <= 1e-11, max|dG| <= 1e-9, sign
exact.  Mixed paths: relative log-det error <= 1e-8 (the target of the mixed-precision
form), max|dG| <= 1e-6 (the bar for the FP32-class forms; several int8-slice tests below
hold tighter ones).  The int8-slice path meets it; the FP32 and bf16 split forms are
asserted against the same 1e-8 bar under a strict xfail (their FP32 matrix-core
accumulation leaves an error floor above it), with the measured error printed."""

import numpy as np
import pytest

import oracle
from synth import workload_item, workload_models, gen

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

import paper_1802_06177_amd as slmc  # noqa: E402

DEV = "cuda:0"
T5_REL, T5_G = 1e-8, 1e-6     # mixed-precision bars: relative log-det, max |dG|


def _E(md):
    return oracle.expk(oracle.hopping_matrix(md["Lx"], md["Ly"], md["t"], md["mu"]), md["dtau"])


def _ref(md, x):
    return oracle.logdet_green(_E(md), x, md["dtau"], md["lam"], md["n_s"])


def _run(md, xs, prec="fp64", resid=0, chunk=0, want_g=True):
    print("case: %dx%d Ltau=%d n_s=%d items=%d prec=%s chunk=%d resid=%d" %
          (md["Lx"], md["Ly"], md["Ltau"], md["n_s"], len(xs), prec, chunk, resid), flush=True)
    m = slmc.model_from_dict(md)
    x = torch.tensor(np.stack(xs), dtype=torch.float64, device=DEV)
    opt = slmc.options(prec, resid, chunk)
    if want_g:
        ld, sg, G, st = slmc.green(m, x, opt)
        torch.cuda.synchronize()
        return ld.cpu().numpy(), sg.cpu().numpy(), G.cpu().numpy(), st.cpu().numpy()
    ld, sg, st = slmc.logdet(m, x, opt)
    torch.cuda.synchronize()
    return ld.cpu().numpy(), sg.cpu().numpy(), None, st.cpu().numpy()


def _check(md, xs, out, rel_tol, g_tol, sign=True):
    ld, sg, G, st = out
    worst_rel, worst_g = 0.0, 0.0
    for k, x in enumerate(xs):
        ref, rs, rG = _ref(md, x)
        assert st[k] == 0
        rel = abs(ld[k] - ref) / abs(ref)
        worst_rel = max(worst_rel, rel)
        if sign:
            assert sg[k] == rs, (k, sg[k], rs)
        if G is not None:
            worst_g = max(worst_g, float(np.max(np.abs(G[k] - rG))))
    print("  max rel logdet %.3e  max|dG| %.3e" % (worst_rel, worst_g), flush=True)
    assert worst_rel <= rel_tol
    assert worst_g <= g_tol
    return worst_rel, worst_g


def _md(L, Ltau, n_s, lam=1.5, Ly=None, mu=0.0):
    return dict(Lx=L, Ly=Ly or L, Ltau=Ltau, n_s=n_s, t=1.0, mu=mu, dtau=0.1, lam=lam,
                omega0=1.0, c_kin=0.5)


# ------------------------------------------------------------------------- FP64 path

def test_fp64_workload_4x4_all_items():
    md = workload_models("W1")[0]
    xs = [workload_item("W1", b)[1] for b in range(64)]
    _check(md, xs, _run(md, xs), 1e-11, 1e-9)


@pytest.mark.parametrize("Lx,Ly,Ltau,n_s,lam", [(2, 2, 12, 4, 3.0), (2, 3, 10, 3, 2.5),
                                                (4, 4, 37, 10, 1.5), (4, 4, 20, 1, 1.5),
                                                (4, 4, 20, 20, 1.5), (6, 6, 30, 7, 2.0),
                                                (6, 4, 24, 5, 1.0), (10, 10, 40, 8, 1.5)])
def test_fp64_shapes_ragged_and_padded(Lx, Ly, Ltau, n_s, lam):
    md = _md(Lx, Ltau, n_s, lam, Ly=Ly, mu=0.1)
    g = gen(99, Lx * 1000 + Ly * 100 + Ltau)
    xs = [g.normal(0.0, 1.5, size=(Ltau, Lx * Ly)) for _ in range(6)]
    _check(md, xs, _run(md, xs), 1e-11, 1e-9)


def test_fp64_negative_determinants_keep_their_sign():
    md = _md(2, 40, 5, 3.0)
    g = gen(98, 1)
    xs = [g.normal(0.0, 3.0, size=(40, 4)) for _ in range(40)]
    out = _run(md, xs)
    refs = [_ref(md, x)[1] for x in xs]
    assert min(refs) < 0 < max(refs)
    _check(md, xs, out, 1e-11, 1e-9)


def test_fp64_workload_8x8_subset():
    md = workload_models("W2")[0]
    xs = [workload_item("W2", b)[1] for b in range(0, 256, 32)]
    _check(md, xs, _run(md, xs), 1e-11, 1e-9)


def test_fp64_closed_form_staggered_16x16():
    # the 16 staggered fields of the 16x16 workload (noiseless) against the momentum-pair
    # closed form, on the full size
    import pins
    md = workload_models("W4", 2)[0]
    items = [128, 129]
    xs = [workload_item("W4", b, 2)[1] for b in items]
    ld, sg, _, st = _run(md, xs, want_g=False)
    for k, b in enumerate(items):
        x0 = xs[k][0, 0]
        ref = pins.staggered_logdet(16, 16, 1.0, 0.0, 0.1, md["lam"], x0, md["Ltau"])
        assert st[k] == 0 and sg[k] == 1
        assert abs(ld[k] - ref) <= 1e-11 * abs(ref), (ld[k], ref)


def test_fp64_free_fermion_16x16():
    import pins
    md = workload_models("W4")[0]
    ld, sg, G, st = _run(md, [np.zeros((160, 256))])
    ref = pins.free_logdet(16, 16, 1.0, 0.0, 16.0)
    assert abs(ld[0] - ref) <= 1e-11 * ref
    assert np.max(np.abs(G[0] - pins.free_green(16, 16, 1.0, 0.0, 16.0))) < 1e-9


@pytest.mark.parametrize("Lx,Ly,Ltau,n_s", [(16, 17, 16, 8), (18, 18, 16, 8), (20, 20, 24, 8),
                                             (21, 21, 18, 6)])
def test_fp64_largest_lattices(Lx, Ly, Ltau, n_s):
    # N = 272 and 324 (padded to 336): the QR's trailing update by wave pairs at its smallest
    # size (17 row blocks, halves of 9 and 8) and at an odd split (21: 11 and 10); N = 400
    # (its largest size, 13 and 12), and N = 441 (padded to 448, the largest size the library
    # accepts)
    md = _md(Lx, Ltau, n_s, 1.5, Ly=Ly)
    g = gen(95, Lx * Ly)
    xs = [g.normal(0.0, 1.0, size=(Ltau, Lx * Ly)) for _ in range(2)]
    _check(md, xs, _run(md, xs), 1e-11, 1e-9)


def test_fp64_full_size_16x16_sampled_items():
    md = workload_models("W4", 1)[0]
    xs = [workload_item("W4", b, 1)[1] for b in (0, 77)]
    _check(md, xs, _run(md, xs), 1e-11, 1e-9)


def test_uneven_batch_one_call():
    # three lattice sizes in one call, packed, items interleaved across models
    mds = [_md(4, 40, 10), _md(6, 30, 10), _md(8, 80, 10)]
    models = [slmc.model_from_dict(d) for d in mds]
    order = [0, 1, 2, 0, 2, 1, 1, 0]
    g = gen(97, 5)
    xs = [g.normal(size=(mds[k]["Ltau"], mds[k]["Lx"] ** 2)) for k in order]
    x_off = np.cumsum([0] + [x.size for x in xs[:-1]])
    g_sizes = [mds[k]["Lx"] ** 4 for k in order]
    g_off = np.cumsum([0] + g_sizes[:-1])
    x = torch.tensor(np.concatenate([a.ravel() for a in xs]), dtype=torch.float64, device=DEV)
    G = torch.zeros(int(sum(g_sizes)), dtype=torch.float64, device=DEV)
    ld, sg, G, st = slmc.green(models, x, slmc.options(), model_idx=order, x_off=x_off,
                               g_off=g_off, n_items=len(order), G=G)
    torch.cuda.synchronize()
    ld, sg, Gh, st = ld.cpu().numpy(), sg.cpu().numpy(), G.cpu().numpy(), st.cpu().numpy()
    for j, k in enumerate(order):
        ref, rs, rG = _ref(mds[k], xs[j])
        N = mds[k]["Lx"] ** 2
        Gj = Gh[g_off[j]:g_off[j] + N * N].reshape(N, N)
        assert st[j] == 0 and sg[j] == rs
        assert abs(ld[j] - ref) <= 1e-11 * abs(ref)
        assert np.max(np.abs(Gj - rG)) < 1e-9


@pytest.mark.parametrize("prec", ["int8x5", "bf16x3", "fp64"])
@pytest.mark.parametrize("Ltau,n_s", [(16, 8), (24, 8), (32, 8), (20, 5), (18, 8)])
def test_few_blocks_overlapped_match_serial_bitwise(prec, Ltau, n_s):
    # 2, 3 and 4 stabilization blocks (and a short last block): the step-by-step release of
    # the side work and the reuse of the three QR output buffers at their smallest counts
    md = _md(8, Ltau, n_s)
    g = gen(99, Ltau + n_s)
    xs = [g.normal(size=(Ltau, 64)) for _ in range(3)]
    m = slmc.model_from_dict(md)
    x = torch.tensor(np.stack(xs), dtype=torch.float64, device=DEV)
    print("case: 8x8 Ltau=%d n_s=%d prec=%s overlapped vs serial" % (Ltau, n_s, prec), flush=True)
    outs = []
    for serial in (False, True):
        ld, sg, G, st = slmc.green(m, x, slmc.options(prec, 1, serial=serial))
        torch.cuda.synchronize()
        outs.append((ld.cpu().numpy(), sg.cpu().numpy(), G.cpu().numpy(), st.cpu().numpy()))
    assert np.all(outs[0][3] == 0)
    for u, v in zip(outs[0], outs[1]):
        assert np.array_equal(u, v)
    bar = 1e-11 if prec == "fp64" else (1e-8 if prec == "int8x5" else 1e-3)
    for k in range(3):
        ref = _ref(md, xs[k])[0]
        assert abs(outs[0][0][k] - ref) <= bar * abs(ref)


@pytest.mark.parametrize("prec", ["fp64", "int8x5"])
def test_packed_groups_overlapped_match_serial_bitwise(prec):
    # six lattice sizes in one call, items interleaved (item tables go into the workspace);
    # two calls back to back on one workspace with different packings, no synchronization
    # between them, overlapped schedule against the serial one (everything in order on the
    # caller's stream); then one item of each size against the oracle
    mds = [_md(4, 20, 5), _md(6, 30, 5), _md(8, 24, 8), _md(4, 16, 4, Ly=6), _md(10, 20, 10),
           _md(12, 24, 6)]
    models = [slmc.model_from_dict(d) for d in mds]
    g = gen(98, 6)
    packs = []
    for order in ([0, 1, 2, 3, 4, 5, 5, 4, 3, 2, 1, 0], [5, 3, 1, 0, 2, 4, 1]):
        xs = [g.normal(size=(mds[k]["Ltau"], mds[k]["Lx"] * mds[k]["Ly"])) for k in order]
        x_off = np.cumsum([0] + [a.size for a in xs[:-1]])
        g_sizes = [(mds[k]["Lx"] * mds[k]["Ly"]) ** 2 for k in order]
        g_off = np.cumsum([0] + g_sizes[:-1])
        x = torch.tensor(np.concatenate([a.ravel() for a in xs]), dtype=torch.float64, device=DEV)
        packs.append((order, x, x_off, g_off, int(sum(g_sizes))))
    opt0 = slmc.options(prec, 1)
    nbytes = max(slmc.workspace_bytes(models, len(o), opt0, model_idx=o, x_off=xo, g_off=go)
                 for o, _, xo, go, _ in packs)
    ws = torch.empty(nbytes, dtype=torch.uint8, device=DEV)
    res = {}
    for serial in (True, False):
        print("case: packed six sizes, prec=%s serial=%s" % (prec, serial), flush=True)
        opt = slmc.options(prec, 1, serial=serial)
        outs = [slmc.green(models, x, opt, model_idx=o, x_off=xo, g_off=go, n_items=len(o),
                           G=torch.empty(ng, dtype=torch.float64, device=DEV), ws=ws)
                for o, x, xo, go, ng in packs]
        torch.cuda.synchronize()
        res[serial] = [[t.cpu().numpy() for t in r] for r in outs]
    for a, b in zip(res[True], res[False]):
        assert np.all(a[3] == 0) and np.all(b[3] == 0)
        for u, v in zip(a, b):
            assert np.array_equal(u, v)
    o, x, xo, go, _ = packs[0]
    xh = x.cpu().numpy()
    ld, _, Gh, _ = res[False][0]
    bar = 1e-11 if prec == "fp64" else 1e-8
    for j in range(6):
        md = mds[o[j]]
        N = md["Lx"] * md["Ly"]
        xj = xh[xo[j]:xo[j] + md["Ltau"] * N].reshape(md["Ltau"], N)
        ref, _, rG = _ref(md, xj)
        assert abs(ld[j] - ref) <= bar * abs(ref)
        assert np.max(np.abs(Gh[go[j]:go[j] + N * N].reshape(N, N) - rG)) < 1e3 * bar


def test_nonfinite_input_flags_only_that_item():
    md = _md(4, 20, 5)
    g = gen(96, 1)
    xs = [g.normal(size=(20, 16)) for _ in range(3)]
    xs[1] = xs[1].copy()
    xs[1][3, 5] = np.nan
    ld, sg, G, st = _run(md, xs)
    assert st[1] == 5 and np.isnan(ld[1])
    assert st[0] == 0 and st[2] == 0
    for k in (0, 2):
        assert abs(ld[k] - _ref(md, xs[k])[0]) <= 1e-11 * abs(ld[k])


def test_run_twice_bitwise_identical():
    md = workload_models("W2")[0]
    xs = [workload_item("W2", b)[1] for b in range(4)]
    a = _run(md, xs, prec="fp32", chunk=1)
    b = _run(md, xs, prec="fp32", chunk=1)
    assert np.array_equal(a[0], b[0]) and np.array_equal(a[2], b[2])


@pytest.mark.parametrize("prec", ["fp64", "fp32", "int8x5", "bf16x3"])
def test_overlapped_and_serial_schedules_are_bitwise_identical(prec):
    # segment products and V updates on the library's side streams (default; all queued up
    # front for FP64 and FP32, released step by step for int8x5 and bf16x3) or everything
    # on the caller's stream
    md = workload_models("W2")[0]
    xs = [workload_item("W2", b)[1] for b in range(5)]
    m = slmc.model_from_dict(md)
    x = torch.tensor(np.stack(xs), dtype=torch.float64, device=DEV)
    outs = []
    for serial in (False, True, False):
        ld, sg, G, st = slmc.green(m, x, slmc.options(prec, 1, 1, serial=serial))
        torch.cuda.synchronize()
        outs.append((ld.cpu().numpy(), G.cpu().numpy()))
    for o in outs[1:]:
        assert np.array_equal(o[0], outs[0][0]) and np.array_equal(o[1], outs[0][1])


def test_residual_step_does_not_degrade_G():
    md = workload_models("W2")[0]
    xs = [workload_item("W2", b)[1] for b in range(3)]
    g0 = _check(md, xs, _run(md, xs, resid=0), 1e-11, 1e-9)[1]
    g1 = _check(md, xs, _run(md, xs, resid=1), 1e-11, 1e-9)[1]
    assert g1 <= 2 * g0 + 1e-14


def test_logdet_only_equals_green_logdet():
    md = workload_models("W1")[0]
    xs = [workload_item("W1", b)[1] for b in range(8)]
    a = _run(md, xs, want_g=False)
    b = _run(md, xs)
    assert np.array_equal(a[0], b[0]) and np.array_equal(a[1], b[1])


# ------------------------------------------------------------------------- mixed paths
# Every precision form is held to the same 1e-8 relative log-det bar.  The FP32 matrix
# cores round while they accumulate, which leaves a coherent error of a few 1e-8 (FP32 with
# FP64 promotion every k-step) up to 1e-5 (bf16x3) even with the compensation of E's
# rounding; those forms fail the bar and are marked as expected failures (strict: a pass
# would flag that the floor moved).  The worst error is printed before the assertion.

_FP32_FLOOR = "FP32 matrix-core accumulation floor: measured error above the 1e-8 target"


@pytest.mark.parametrize("prec,chunk", [
    pytest.param("fp32", 1, marks=pytest.mark.xfail(strict=True, raises=AssertionError, reason=_FP32_FLOOR)),
    pytest.param("fp32", 4, marks=pytest.mark.xfail(strict=True, raises=AssertionError, reason=_FP32_FLOOR)),
    pytest.param("fp32", 0, marks=pytest.mark.xfail(strict=True, raises=AssertionError, reason=_FP32_FLOOR)),
    pytest.param("fp32plain", 1, marks=pytest.mark.xfail(strict=True, raises=AssertionError, reason=_FP32_FLOOR)),
    pytest.param("bf16x6", 0, marks=pytest.mark.xfail(strict=True, raises=AssertionError, reason=_FP32_FLOOR)),
    pytest.param("bf16x3", 0, marks=pytest.mark.xfail(strict=True, raises=AssertionError, reason=_FP32_FLOOR)),
    ("int8x5", 0)])
def test_mixed_variants_meet_1e8_8x8(prec, chunk):
    md = workload_models("W2")[0]
    xs = [workload_item("W2", b)[1] for b in range(0, 256, 64)]
    _check(md, xs, _run(md, xs, prec=prec, chunk=chunk), T5_REL, T5_G)


def test_fp32_compensation_of_E_reduces_error():
    md = workload_models("W2")[0]
    xs = [workload_item("W2", b)[1] for b in range(0, 256, 64)]
    refs = [_ref(md, x)[0] for x in xs]
    plain = _run(md, xs, prec="fp32plain", chunk=1)[0]
    comp = _run(md, xs, prec="fp32", chunk=1)[0]
    ep = max(abs(plain[k] - refs[k]) / abs(refs[k]) for k in range(len(xs)))
    ec = max(abs(comp[k] - refs[k]) / abs(refs[k]) for k in range(len(xs)))
    print("  plain %.3e  compensated %.3e" % (ep, ec))
    assert ec < 0.6 * ep


@pytest.mark.parametrize("prec", [
    pytest.param("fp32", marks=pytest.mark.xfail(strict=True, raises=AssertionError, reason=_FP32_FLOOR)),
    pytest.param("bf16x3", marks=pytest.mark.xfail(strict=True, raises=AssertionError, reason=_FP32_FLOOR))])
def test_split_forms_full_size_16x16_meet_1e8(prec):
    md = workload_models("W4", 1)[0]
    xs = [workload_item("W4", b, 1)[1] for b in (3,)]
    _check(md, xs, _run(md, xs, prec=prec, chunk=1 if prec == "fp32" else 0, resid=1), T5_REL, T5_G)


# ------------------------------------------------------------------------- int8 slices
# The int8 split accumulates exactly; its error comes only from cutting E and the panels
# into 5 slices of 7 bits (about 2^-36 relative per product), so it must meet the 1e-8
# relative log-det target at the full 16x16 size and on padded / ragged shapes.

def test_int8x5_full_size_16x16_meets_1e8():
    md = workload_models("W4", 1)[0]
    xs = [workload_item("W4", b, 1)[1] for b in (0, 77)]
    _check(md, xs, _run(md, xs, prec="int8x5", resid=1), 1e-8, 1e-7)


@pytest.mark.parametrize("lam_idx", [0, 2])
def test_int8x5_16x16_other_couplings(lam_idx):
    md = workload_models("W4", lam_idx)[0]
    xs = [workload_item("W4", b, lam_idx)[1] for b in (3,)]
    _check(md, xs, _run(md, xs, prec="int8x5", resid=1), 1e-8, 1e-7)


@pytest.mark.parametrize("Lx,Ly,Ltau,n_s", [(2, 3, 10, 3), (6, 6, 30, 7), (10, 10, 40, 8),
                                             (12, 12, 36, 10), (18, 18, 16, 8), (20, 20, 16, 8),
                                             (4, 4, 20, 1)])
def test_int8x5_ragged_and_padded_shapes(Lx, Ly, Ltau, n_s):
    md = _md(Lx, Ltau, n_s, 1.5, Ly=Ly, mu=0.1)
    g = gen(94, Lx * 1000 + Ly * 100 + Ltau)
    xs = [g.normal(0.0, 1.5, size=(Ltau, Lx * Ly)) for _ in range(3)]
    _check(md, xs, _run(md, xs, prec="int8x5"), 1e-9, 1e-8)


# E is a function of the displacement only, so its row blocks repeat (columns rotated) every
# lcm(16, Lx) rows when N is a multiple of 16; the int8 kernel then keeps the base rows'
# slices in LDS.  Integer sums are exact, so the result must equal the streaming mode's
# bit for bit, and both must meet the oracle bar.
# (16x16, 8x8, 16x8 and 16x12 also take the register variant: one base row block, Np a
# multiple of 64, each wave's few distinct A operands held in registers)
@pytest.mark.parametrize("Lx,Ly,Ltau,n_s", [(16, 16, 40, 8), (12, 12, 36, 10), (8, 6, 24, 6),
                                             (4, 4, 20, 5), (16, 28, 16, 8), (8, 10, 20, 7),
                                             (8, 8, 24, 6), (16, 8, 20, 5), (16, 12, 16, 8)])
def test_int8x5_lds_base_rows_equal_streamed_bitwise(Lx, Ly, Ltau, n_s):
    md = _md(Lx, Ltau, n_s, 1.5, Ly=Ly, mu=0.1)
    g = gen(95, Lx * 1000 + Ly * 100 + Ltau)
    xs = [g.normal(0.0, 1.5, size=(Ltau, Lx * Ly)) for _ in range(3)]
    print("case: %dx%d Ltau=%d n_s=%d int8x5 LDS base rows vs streamed E" % (Lx, Ly, Ltau, n_s), flush=True)
    m = slmc.model_from_dict(md)
    x = torch.tensor(np.stack(xs), dtype=torch.float64, device=DEV)
    outs = []
    for stream_e in (False, True):
        r = slmc.green(m, x, slmc.options("int8x5", 1, 0, stream_e=stream_e))
        torch.cuda.synchronize()
        outs.append([t.cpu().numpy() for t in r])
    for a, b in zip(outs[0], outs[1]):
        assert np.array_equal(a, b)
    _check(md, xs[:1], [o[:1] for o in outs[0]], 1e-9, 1e-8)


def test_int8x5_negative_determinants_keep_their_sign():
    md = _md(2, 40, 5, 3.0)
    g = gen(98, 1)
    xs = [g.normal(0.0, 3.0, size=(40, 4)) for _ in range(40)]
    out = _run(md, xs, prec="int8x5", resid=1)
    refs = [_ref(md, x)[1] for x in xs]
    assert min(refs) < 0 < max(refs)
    _check(md, xs, out, T5_REL, T5_G)


def test_int8x5_nonfinite_input_flags_only_that_item():
    md = _md(8, 24, 6)
    g = gen(96, 2)
    xs = [g.normal(size=(24, 64)) for _ in range(3)]
    xs[1] = xs[1].copy()
    xs[1][7, 9] = np.inf
    ld, sg, G, st = _run(md, xs, prec="int8x5", resid=1)
    assert st[1] == 5 and np.isnan(ld[1])
    assert st[0] == 0 and st[2] == 0
    for k in (0, 2):
        ref = _ref(md, xs[k])
        assert abs(ld[k] - ref[0]) <= T5_REL * abs(ref[0])
        assert np.max(np.abs(G[k] - ref[2])) <= T5_G


def test_int8x5_staggered_closed_form_16x16():
    import pins
    md = workload_models("W4", 2)[0]
    xs = [workload_item("W4", b, 2)[1] for b in (128, 129)]
    ld, sg, _, st = _run(md, xs, prec="int8x5", want_g=False)
    for k, x in enumerate(xs):
        ref = pins.staggered_logdet(16, 16, 1.0, 0.0, 0.1, md["lam"], x[0, 0], md["Ltau"])
        assert st[k] == 0 and sg[k] == 1
        assert abs(ld[k] - ref) <= 1e-8 * abs(ref), (ld[k], ref)


# ------------------------------------------------------------------------- packed uneven batch
# The uneven workload: 32 fields for each of L = 8, 12, 16, 20 (Ltau = 10 L, n_s = 10) in one
# packed call, items interleaved across the four models; sampled items against the oracle.

@pytest.mark.parametrize("prec,rel_bar,g_bar", [("fp64", 1e-11, 1e-9), ("int8x5", 1e-8, 1e-7)])
def test_uneven_workload_packed_sampled(prec, rel_bar, g_bar):
    mds = workload_models("W5")
    models = [slmc.model_from_dict(d) for d in mds]
    items = list(range(128))
    order = [items[(7 * k) % 128] for k in range(128)]          # interleave the sizes
    xs, midx = [], []
    for b in order:
        mi, x = workload_item("W5", b)
        xs.append(x)
        midx.append(mi)
    x_off = np.cumsum([0] + [x.size for x in xs[:-1]])
    g_sizes = [(mds[k]["Lx"] * mds[k]["Ly"]) ** 2 for k in midx]
    g_off = np.cumsum([0] + g_sizes[:-1])
    x = torch.tensor(np.concatenate([a.ravel() for a in xs]), dtype=torch.float64, device=DEV)
    G = torch.zeros(int(sum(g_sizes)), dtype=torch.float64, device=DEV)
    print("case: uneven W5 packed, 128 items, prec=%s" % prec, flush=True)
    ld, sg, G, st = slmc.green(models, x, slmc.options(prec, 1), model_idx=midx, x_off=x_off,
                               g_off=g_off, n_items=len(order), G=G)
    torch.cuda.synchronize()
    ld, sg, Gh, st = ld.cpu().numpy(), sg.cpu().numpy(), G.cpu().numpy(), st.cpu().numpy()
    assert np.all(st == 0)
    # one sampled item per size class (the oracle at L = 20 takes a few seconds)
    seen = set()
    for j, mi in enumerate(midx):
        if mi in seen:
            continue
        seen.add(mi)
        ref, rs, rG = _ref(mds[mi], xs[j])
        N = mds[mi]["Lx"] * mds[mi]["Ly"]
        Gj = Gh[g_off[j]:g_off[j] + N * N].reshape(N, N)
        assert sg[j] == rs
        assert abs(ld[j] - ref) <= rel_bar * abs(ref), (mi, ld[j], ref)
        assert np.max(np.abs(Gj - rG)) <= g_bar
    assert seen == {0, 1, 2, 3}
