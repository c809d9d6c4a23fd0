"""The entry point that allocates nothing (slmc_green_noalloc) against slmc_green: same
fields, same results (the same kernels; the serial schedule gives the results of the
overlapped one bit for bit), on two calls in a row, the second with a smaller input of
another model; a batch beyond the static scratch is refused before anything is enqueued."""

import numpy as np
import pytest

import oracle
from synth import workload_item, workload_models, gen

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

import paper_1802_06177_amd as slmc  # noqa: E402
from paper_1802_06177_amd import _abi  # noqa: E402

DEV = "cuda:0"


def _np(r):
    return [t.cpu().numpy() for t in r]


@pytest.mark.parametrize("prec", ["fp64", "int8x5"])
def test_noalloc_matches_green_on_two_calls(prec):
    resid = 0 if prec == "fp64" else 1
    opt = slmc.options(prec, resid)
    # call 1: 40 fields of the 8x8, Ltau 80 workload; call 2: 9 fields of the 4x4 one
    cases = []
    md1 = workload_models("W2")[0]
    cases.append((md1, [workload_item("W2", b)[1] for b in range(40)]))
    md2 = workload_models("W1")[0]
    cases.append((md2, [workload_item("W1", b)[1] for b in (0, 5, 9, 17, 33, 47, 50, 58, 63)]))
    xs_dev = []
    outs = []
    for md, xs in cases:
        print("case: noalloc %dx%d Ltau=%d items=%d prec=%s" % (md["Lx"], md["Ly"], md["Ltau"], len(xs), prec),
              flush=True)
        m = slmc.model_from_dict(md)
        x = torch.tensor(np.stack(xs), dtype=torch.float64, device=DEV)
        xs_dev.append(x)
        outs.append(_np(slmc.green_noalloc(m, x, opt)))
    torch.cuda.synchronize()
    for (md, xs), x, got in zip(cases, xs_dev, outs):
        m = slmc.model_from_dict(md)
        ref = _np(slmc.green(m, x, opt))
        torch.cuda.synchronize()
        assert np.all(got[3] == 0)
        for a, b in zip(got, ref):
            assert np.array_equal(a, b)
        # and the first item against the oracle at the path's bar
        E = oracle.expk(oracle.hopping_matrix(md["Lx"], md["Ly"], md["t"], md["mu"]), md["dtau"])
        ld, s, G = oracle.logdet_green(E, xs[0], md["dtau"], md["lam"], md["n_s"])
        bar = (1e-11, 1e-9) if prec == "fp64" else (1e-8, 1e-6)
        assert abs(got[0][0] - ld) <= bar[0] * abs(ld) and got[1][0] == s
        assert np.max(np.abs(got[2][0] - G)) <= bar[1]


def test_noalloc_logdet_only_and_repeat_same_model():
    md = workload_models("W1")[0]
    m = slmc.model_from_dict(md)
    x = torch.tensor(np.stack([workload_item("W1", b)[1] for b in range(16)]), dtype=torch.float64,
                     device=DEV)
    a = _np(slmc.green_noalloc(m, x, slmc.options("fp64"), want_g=False))
    b = _np(slmc.green_noalloc(m, x[:7].contiguous(), slmc.options("fp64"), want_g=False))
    ref = _np(slmc.logdet(m, x, slmc.options("fp64")))
    torch.cuda.synchronize()
    assert np.array_equal(a[0], ref[0]) and np.array_equal(a[1], ref[1])
    assert np.array_equal(b[0], ref[0][:7]) and np.array_equal(b[1], ref[1][:7])


def test_noalloc_refuses_a_batch_beyond_the_scratch():
    md = workload_models("W4", 1)[0]
    m = slmc.model_from_dict(md)
    n = 1
    while slmc.workspace_bytes(m, n + 1) <= _abi.SLMC_NOALLOC_WORKSPACE_BYTES:
        n += 1
    x = torch.zeros((n + 1, md["Ltau"], 256), dtype=torch.float64, device=DEV)
    with pytest.raises(slmc.SlmcError) as e:
        slmc.green_noalloc(m, x)
    assert e.value.code == _abi.SLMC_E_WORKSPACE
