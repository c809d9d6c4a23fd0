"""HIP-graph capture of one evaluation call (single model): the library forks its side
streams from the caller's stream with events and joins them back, clears with a kernel
rather than a memset and does no host synchronization on this path, so the whole call can
be captured and replayed.  Every replay is checked bitwise against the eager result, with
eager calls and synchronizations between the replays."""

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
