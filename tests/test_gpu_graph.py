"""HIP-graph capture of one evaluation call (single model, and a packed call of two models at
constant strides) and of a whole SLMC step: the
library forks its side streams from the caller's stream with events and joins them back,
clears with a kernel rather than a memset and does no host synchronization on these paths,
so the calls can be captured and replayed.  Every replay is checked bitwise against the
eager result, with eager calls and synchronizations between the replays."""

import numpy as np
import pytest

from synth import workload_item, workload_models

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

import paper_1802_06177_amd as slmc  # noqa: E402

DEV = "cuda:0"


def _host(out):
    return [t.cpu().numpy().copy() for t in out]


@pytest.mark.parametrize("prec", ["fp64", "int8x5"])
def test_green_call_replays_from_a_captured_graph(prec):
    md = workload_models("W2")[0]
    m = slmc.model_from_dict(md)
    N, B = md["Lx"] * md["Ly"], 6
    xa = np.stack([workload_item("W2", b)[1] for b in range(B)])
    xb = np.stack([workload_item("W2", b)[1] for b in range(B, 2 * B)])
    opt = slmc.options(prec, 1)
    nbytes = slmc.workspace_bytes(m, B, opt)
    # eager references, on buffers of their own (this also creates the library's streams)
    ws_e = torch.empty(nbytes, dtype=torch.uint8, device=DEV)
    refs = []
    for xs in (xa, xb):
        xe = torch.tensor(xs, dtype=torch.float64, device=DEV)
        refs.append(_host(slmc.green(m, xe, opt, G=torch.empty((B, N, N), dtype=torch.float64, device=DEV),
                                     ws=ws_e)))
    torch.cuda.synchronize()
    assert np.all(refs[0][3] == 0) and np.all(refs[1][3] == 0)
    # capture
    x = torch.tensor(xa, dtype=torch.float64, device=DEV)
    G = torch.empty((B, N, N), dtype=torch.float64, device=DEV)
    ws = torch.empty(nbytes, dtype=torch.uint8, device=DEV)
    print("case: capture green W2 x%d prec=%s" % (B, prec), flush=True)
    graph = torch.cuda.CUDAGraph()
    with torch.cuda.graph(graph):
        out = slmc.green(m, x, opt, G=G, ws=ws)
    torch.cuda.synchronize()
    for r, xs in enumerate((xa, xb, xa, xb)):
        print("case: replay %d" % r, flush=True)
        x.copy_(torch.tensor(xs, dtype=torch.float64, device=DEV))
        graph.replay()
        torch.cuda.synchronize()
        got = _host(out)
        want = refs[r % 2]
        for u, v in zip(got, want):
            assert np.array_equal(u, v)
        # eager work between the replays, on the library's streams too
        slmc.green(m, torch.tensor(xb, dtype=torch.float64, device=DEV), opt,
                   G=torch.empty((B, N, N), dtype=torch.float64, device=DEV), ws=ws_e)
        torch.cuda.synchronize()


@pytest.mark.parametrize("prec", ["fp64", "int8x5"])
def test_slmc_step_replays_from_a_captured_graph(prec):
    # the whole SLMC step (copy, sweeps and cluster moves, log-det chain, accept) captured
    # once and replayed step after step: the proposal index lives in device memory and
    # advances with every replay.  Each replay must equal the eager step of the same index,
    # and the eager step the explicit calls (propose + cumulative accept) of that index.
    from synth import gen, eff_coefficients
    md = dict(Lx=8, Ly=8, Ltau=40, n_s=10, t=1.0, mu=0.0, dtau=0.1, lam=1.5, omega0=1.0, c_kin=0.5)
    m = slmc.model_from_dict(md)
    eff = slmc.eff_model(**eff_coefficients(3, 0, 1.5, delta=2.5))   # large moves: some rejected
    C, K, seed, c0 = 6, 4, 2718, 40
    x0 = gen(701, 0).normal(0.0, 1.0, size=(C, 40, 64))
    opt = slmc.options(prec, 1)
    from paper_1802_06177_amd import _abi
    import ctypes as Cc
    nbytes = _abi.lib().slmc_accept_workspace_bytes(Cc.byref(m), C, Cc.byref(opt))

    def state():
        xc = torch.tensor(x0, dtype=torch.float64, device=DEV)
        lw, st = slmc.log_weight(m, xc, opt)
        ee = slmc.eff_energy(m, eff, xc)
        return xc, torch.empty_like(xc), lw, ee

    # explicit calls with explicit proposal indices
    xe, xpe, lwe, eee = state()
    explicit = []
    for k in range(K):
        xpe.copy_(xe)
        slmc.eff_propose(m, eff, xpe, 1, 2, seed, c0 + k)
        acc, lr, st = slmc.cumulative_accept(m, eff, xe, xpe, lwe, eee, seed, c0 + k, opt)
        explicit.append(_host([xe, lwe, eee, acc, lr]))
    # eager steps
    xs_, xps, lws, ees = state()
    cnt = torch.tensor([c0], dtype=torch.int64, device=DEV)
    ws_e = torch.empty(nbytes, dtype=torch.uint8, device=DEV)
    eager = []
    for k in range(K):
        out = slmc.step(m, eff, xs_, xps, lws, ees, 1, 2, seed, cnt, opt, ws=ws_e)
        eager.append(_host([xs_, lws, ees, out["accepted"], out["log_ratio"]]))
        assert np.all(out["status"].cpu().numpy() == 0)
    assert int(cnt.item()) == c0 + K
    torch.cuda.synchronize()
    for a, b in zip(explicit, eager):
        for u, v in zip(a, b):
            assert np.array_equal(u, v)
    assert 0 < sum(int(e[3].sum()) for e in eager) < C * K     # both decisions occur
    # capture one step, replay K times
    xg, xpg, lwg, eeg = state()
    cg = torch.tensor([c0], dtype=torch.int64, device=DEV)
    ws = torch.empty(nbytes, dtype=torch.uint8, device=DEV)
    outg = {"accepted": torch.empty(C, dtype=torch.uint8, device=DEV),
            "log_ratio": torch.empty(C, dtype=torch.float64, device=DEV),
            "status": torch.empty(C, dtype=torch.int32, device=DEV),
            "n_local": torch.empty(C, dtype=torch.int64, device=DEV)}
    torch.cuda.synchronize()
    print("case: capture slmc_step 8x8 Ltau=40 prec=%s" % prec, flush=True)
    graph = torch.cuda.CUDAGraph()
    with torch.cuda.graph(graph):
        slmc.step(m, eff, xg, xpg, lwg, eeg, 1, 2, seed, cg, opt, out=outg, ws=ws)
    torch.cuda.synchronize()
    # capturing ran nothing: the state is still the initial one
    assert int(cg.item()) == c0
    for k in range(K):
        print("case: replay %d" % k, flush=True)
        graph.replay()
        torch.cuda.synchronize()
        got = _host([xg, lwg, eeg, outg["accepted"], outg["log_ratio"]])
        for u, v in zip(got, eager[k]):
            assert np.array_equal(u, v)
        # eager work between the replays
        slmc.step(m, eff, xs_, xps, lws, ees, 1, 2, seed, torch.tensor([999], dtype=torch.int64, device=DEV),
                  opt, ws=ws_e)
        torch.cuda.synchronize()
    assert int(cg.item()) == c0 + K


@pytest.mark.parametrize("prec", ["fp64", "int8x5"])
def test_packed_constant_stride_call_replays_from_a_captured_graph(prec):
    # a packed call of two models whose items are laid out model by model at constant
    # strides: no item table is uploaded and nothing waits on the host, so the call (the
    # larger model's overlapped schedule on the caller's stream, the other model serially
    # on a third library stream) can be captured and replayed
    from synth import gen
    mds = [dict(Lx=8, Ly=8, Ltau=40, n_s=10, t=1.0, mu=0.0, dtau=0.1, lam=1.5, omega0=1.0, c_kin=0.5),
           dict(Lx=4, Ly=6, Ltau=30, n_s=10, t=1.0, mu=0.1, dtau=0.1, lam=1.2, omega0=1.0, c_kin=0.5)]
    models = [slmc.model_from_dict(d) for d in mds]
    counts = [3, 4]
    midx = [0] * counts[0] + [1] * counts[1]
    xs_sz = [d["Ltau"] * d["Lx"] * d["Ly"] for d in mds]
    gs_sz = [(d["Lx"] * d["Ly"]) ** 2 for d in mds]
    x_off = np.cumsum([0] + [xs_sz[k] for k in midx[:-1]])
    g_off = np.cumsum([0] + [gs_sz[k] for k in midx[:-1]])
    nx, ng = int(sum(xs_sz[k] for k in midx)), int(sum(gs_sz[k] for k in midx))
    opt = slmc.options(prec, 1)
    nbytes = slmc.workspace_bytes(models, len(midx), opt, model_idx=midx, x_off=x_off, g_off=g_off)

    def fields(seed):
        return np.concatenate([gen(seed, b).normal(0.0, 1.0, size=xs_sz[k]) for b, k in enumerate(midx)])

    xa, xb = fields(811), fields(812)
    # eager references on buffers of their own
    ws_e = torch.empty(nbytes, dtype=torch.uint8, device=DEV)
    refs = []
    for xv in (xa, xb):
        Ge = torch.empty(ng, dtype=torch.float64, device=DEV)
        out = slmc.green(models, torch.tensor(xv, dtype=torch.float64, device=DEV), opt, model_idx=midx,
                         x_off=x_off, g_off=g_off, n_items=len(midx), G=Ge, ws=ws_e)
        refs.append(_host(out))
    torch.cuda.synchronize()
    assert np.all(refs[0][3] == 0) and np.all(refs[1][3] == 0)
    x = torch.tensor(xa, dtype=torch.float64, device=DEV)
    G = torch.empty(ng, dtype=torch.float64, device=DEV)
    ws = torch.empty(nbytes, dtype=torch.uint8, device=DEV)
    torch.cuda.synchronize()
    print("case: capture packed 8x8 + 4x6 prec=%s" % prec, flush=True)
    graph = torch.cuda.CUDAGraph()
    with torch.cuda.graph(graph):
        out = slmc.green(models, x, opt, model_idx=midx, x_off=x_off, g_off=g_off, n_items=len(midx),
                         G=G, ws=ws)
    torch.cuda.synchronize()
    for r, xv in enumerate((xa, xb, xa, xb)):
        print("case: replay %d" % r, flush=True)
        x.copy_(torch.tensor(xv, dtype=torch.float64, device=DEV))
        graph.replay()
        torch.cuda.synchronize()
        got = _host(out)
        for u, v in zip(got, refs[r % 2]):
            assert np.array_equal(u, v)
        # eager work between the replays
        slmc.green(models, torch.tensor(xb, dtype=torch.float64, device=DEV), opt, model_idx=midx,
                   x_off=x_off, g_off=g_off, n_items=len(midx),
                   G=torch.empty(ng, dtype=torch.float64, device=DEV), ws=ws_e)
        torch.cuda.synchronize()
