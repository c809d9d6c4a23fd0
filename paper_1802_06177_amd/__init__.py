"""MI355X (gfx950) library for the hot path of symmetry-enforced self-learning Monte Carlo
on the 2D Holstein model (arXiv:1802.06177): the fermion weight log|det(1 + B_L...B_1)|
and the equal-time Green's function of a phonon field (SM Eqs. S2, S3), the symmetric
effective model's checkerboard sweeps (Eq. 4) and the cumulative-update acceptance
(Eq. 6).

Everything runs in the HIP kernels behind the C ABI of include/slmc.h; this module only
marshals torch tensors (device memory and the current stream) into those calls.  Inputs
must be CUDA (HIP) float64 tensors; there is no CPU path.
"""

import ctypes as C

import numpy as np

from . import _abi
from ._abi import (SLMC_FP64, SLMC_FP32, SLMC_BF16X3, SLMC_BF16X6, SLMC_FP32_PLAIN, SLMC_INT8X5,
                   SlmcError,
                   Model, Options, Batch, Eff)

__all__ = ["model", "options", "eff_model", "expk", "workspace_bytes", "logdet", "green",
           "eff_energy", "eff_sweep", "eff_wolff", "eff_propose", "log_weight", "cumulative_accept",
           "green_noalloc", "green_slices", "dqmc_sweep", "dqmc_block", "eff_fit", "step",
           "autotune", "tuning", "cache_clear", "SlmcError", "version"]

PRECISIONS = {"fp64": SLMC_FP64, "fp32": SLMC_FP32, "bf16x3": SLMC_BF16X3, "bf16x6": SLMC_BF16X6,
              "fp32plain": SLMC_FP32_PLAIN, "int8x5": SLMC_INT8X5}


def version():
    return _abi.lib().slmc_version()


def model(Lx, Ly, Ltau, n_s, t=1.0, mu=0.0, dtau=0.1, lam=1.5, omega0=1.0, c_kin=0.5):
    """slmc_model of a periodic Lx x Ly lattice with Ltau slices (beta = Ltau dtau)."""
    return Model(int(Lx), int(Ly), int(Ltau), int(n_s), float(t), float(mu), float(dtau),
                 float(lam), float(omega0), float(c_kin))


def model_from_dict(d):
    return model(d["Lx"], d["Ly"], d["Ltau"], d["n_s"], d.get("t", 1.0), d.get("mu", 0.0),
                 d.get("dtau", 0.1), d.get("lam", 1.5), d.get("omega0", 1.0), d.get("c_kin", 0.5))


def options(precision="fp64", residual_steps=0, acc_chunk=0, serial=False, stream_e=False):
    """slmc_options; serial=True keeps every kernel on the caller's stream (no overlap of
    the segment products with the stabilization chain); stream_e=True makes the int8 path
    read all of E in every product instead of an LDS copy of its translation-invariant
    base rows (same result)."""
    p = PRECISIONS[precision] if isinstance(precision, str) else int(precision)
    flags = (_abi.SLMC_FLAG_SERIAL if serial else 0) | (_abi.SLMC_FLAG_STREAM_E if stream_e else 0)
    return Options(p, int(residual_steps), int(acc_chunk), flags)


def eff_model(Jk=0.0, J2=0.0, Jp=0.0, Jp6=0.0, a=0.0, Js=(0.0, 0.0, 0.0), Jt=0.0, delta=0.5):
    e = Eff()
    e.Jk, e.J2, e.Jp, e.Jp6, e.a = float(Jk), float(J2), float(Jp), float(Jp6), float(a)
    for k in range(3):
        e.Js[k] = float(Js[k])
    e.Jt, e.delta = float(Jt), float(delta)
    return e


def expk(m):
    """e^{-dtau K} (host, FP64, N x N) from the library's Fourier construction."""
    N = m.Lx * m.Ly
    out = np.empty((N, N), dtype=np.float64)
    _abi.check(_abi.lib().slmc_expk(C.byref(m), out.ctypes.data_as(C.POINTER(C.c_double))))
    return out


def cache_clear():
    _abi.lib().slmc_cache_clear()


def profile(enable=True):
    """Turns the library's HIP-event kernel timing on or off (see slmc_profile)."""
    _abi.check(_abi.lib().slmc_profile(1 if enable else 0))


def profile_reset():
    _abi.lib().slmc_profile_reset()


def profile_read():
    """{kernel class: (total_ms, launches)} accumulated since the last reset."""
    L = _abi.lib()
    out = {}
    for k in range(8):
        ms, n = C.c_double(), C.c_int64()
        _abi.check(L.slmc_profile_read(k, C.byref(ms), C.byref(n)))
        out[L.slmc_profile_name(k).decode()] = (ms.value, n.value)
    return out


def _torch():
    import torch
    return torch


def _stream(stream):
    torch = _torch()
    s = stream if stream is not None else torch.cuda.current_stream()
    return C.c_void_p(s.cuda_stream)


def _dev_f64(t, name):
    torch = _torch()
    if not isinstance(t, torch.Tensor) or not t.is_cuda or t.dtype != torch.float64:
        raise TypeError("%s must be a float64 tensor on the GPU" % name)
    if not t.is_contiguous():
        raise ValueError("%s must be contiguous" % name)
    return C.c_void_p(t.data_ptr())


def _shape(t, shape, name):
    """The library takes raw pointers and cannot see sizes: every tensor is checked here,
    before its pointer is passed, so a mis-shaped input is a ValueError and never an
    out-of-bounds device access."""
    if tuple(t.shape) != tuple(shape):
        raise ValueError("%s must have shape %s, got %s" % (name, tuple(shape), tuple(t.shape)))


def _fits(t, ends, name):
    """Every packed item [off, off + size) must lie inside t."""
    if len(ends) and int(max(ends)) > t.numel():
        raise ValueError("%s holds %d elements, the packed items need %d"
                         % (name, t.numel(), int(max(ends))))


def _dims(m):
    return m.Ltau, m.Lx * m.Ly


class _BatchArgs:
    """Host-side slmc_batch with the arrays kept alive."""

    def __init__(self, n_items, model_idx=None, x_off=None, g_off=None):
        self._mi = None if model_idx is None else np.ascontiguousarray(model_idx, dtype=np.int32)
        self._xo = None if x_off is None else np.ascontiguousarray(x_off, dtype=np.int64)
        self._go = None if g_off is None else np.ascontiguousarray(g_off, dtype=np.int64)
        P = C.POINTER
        self.batch = Batch(int(n_items),
                           None if self._mi is None else self._mi.ctypes.data_as(P(C.c_int32)),
                           None if self._xo is None else self._xo.ctypes.data_as(P(C.c_int64)),
                           None if self._go is None else self._go.ctypes.data_as(P(C.c_int64)))


def _models_arr(models):
    if isinstance(models, Model):
        models = [models]
    arr = (Model * len(models))(*models)
    return arr, len(models)


# One workspace per (device, stream).  Calls on one stream run in order, so they can share
# a buffer; calls on different streams get different buffers, each allocated while its
# stream is current, so that torch's caching allocator keeps a replaced (smaller) buffer
# away from other streams until the work queued on its own stream has finished with it.
_ws_cache = {}


def _workspace(nbytes, device, stream=None):
    torch = _torch()
    s = stream if stream is not None else torch.cuda.current_stream(device)
    key = (str(device), int(s.cuda_stream))
    buf = _ws_cache.get(key)
    if buf is None or buf.numel() < nbytes:
        _ws_cache.pop(key, None)
        with torch.cuda.stream(s):
            buf = torch.empty(max(int(nbytes), 256), dtype=torch.uint8, device=device)
        _ws_cache[key] = buf
    return buf


def _ws_args(buf):
    if not buf.is_cuda or not buf.is_contiguous():
        raise ValueError("ws must be a contiguous GPU tensor")
    return C.c_void_p(buf.data_ptr()), buf.numel() * buf.element_size()


def workspace_bytes(models, n_items, opt=None, model_idx=None, x_off=None, g_off=None):
    arr, nm = _models_arr(models)
    ba = _BatchArgs(n_items, model_idx, x_off, g_off)
    opt = opt or options()
    return _abi.lib().slmc_workspace_bytes(arr, nm, C.byref(ba.batch), C.byref(opt))


def _check_fermion_shapes(arr, nm, x, n_items, model_idx, x_off, g_off, G):
    mi = np.zeros(n_items, dtype=np.int64) if model_idx is None else np.asarray(model_idx, dtype=np.int64)
    if mi.shape != (n_items,) or (n_items and (mi.min() < 0 or mi.max() >= nm)):
        raise ValueError("model_idx must hold n_items entries in [0, %d)" % nm)
    xs = np.array([arr[k].Ltau * arr[k].Lx * arr[k].Ly for k in range(nm)], dtype=np.int64)[mi]
    gs = np.array([(arr[k].Lx * arr[k].Ly) ** 2 for k in range(nm)], dtype=np.int64)[mi]
    if x_off is None:
        if nm == 1 and x.dim() == 3:
            _shape(x, (n_items,) + _dims(arr[0]), "x")
        else:
            _fits(x, np.cumsum(xs), "x")
    else:
        xo = np.asarray(x_off, dtype=np.int64)
        if xo.shape != (n_items,) or (n_items and xo.min() < 0):
            raise ValueError("x_off must hold n_items non-negative offsets")
        _fits(x, xo + xs, "x")
    if G is not None:
        if g_off is None:
            if nm == 1 and G.dim() == 3:
                N = arr[0].Lx * arr[0].Ly
                _shape(G, (n_items, N, N), "G")
            else:
                _fits(G, np.cumsum(gs), "G")
        else:
            go = np.asarray(g_off, dtype=np.int64)
            if go.shape != (n_items,) or (n_items and go.min() < 0):
                raise ValueError("g_off must hold n_items non-negative offsets")
            _fits(G, go + gs, "G")


def _fermion(models, x, opt, model_idx, x_off, g_off, n_items, want_g, G, stream, ws):
    torch = _torch()
    arr, nm = _models_arr(models)
    if n_items is None:
        if nm != 1 or x.dim() != 3:
            raise ValueError("x must be [items, Ltau, N] for a single model, else pass n_items")
        n_items = x.shape[0]
    if want_g and G is None and nm != 1:
        raise ValueError("pass G for several models")
    _check_fermion_shapes(arr, nm, x, n_items, model_idx, x_off, g_off, G)
    xp = _dev_f64(x, "x")
    opt = opt or options()
    ba = _BatchArgs(n_items, model_idx, x_off, g_off)
    L = _abi.lib()
    need = L.slmc_workspace_bytes(arr, nm, C.byref(ba.batch), C.byref(opt))
    wsp, wsn = _ws_args(ws if ws is not None else _workspace(need, x.device, stream))
    logdet = torch.empty(n_items, dtype=torch.float64, device=x.device)
    sign = torch.empty(n_items, dtype=torch.int8, device=x.device)
    status = torch.empty(n_items, dtype=torch.int32, device=x.device)
    vp = C.c_void_p
    if want_g:
        if G is None:
            N = arr[0].Lx * arr[0].Ly
            G = torch.empty((n_items, N, N), dtype=torch.float64, device=x.device)
        _abi.check(L.slmc_green(arr, nm, C.byref(ba.batch), C.byref(opt), xp,
                                vp(logdet.data_ptr()), vp(sign.data_ptr()), _dev_f64(G, "G"),
                                vp(status.data_ptr()), wsp, wsn, _stream(stream)))
        return logdet, sign, G, status
    _abi.check(L.slmc_logdet(arr, nm, C.byref(ba.batch), C.byref(opt), xp,
                             vp(logdet.data_ptr()), vp(sign.data_ptr()), vp(status.data_ptr()),
                             wsp, wsn, _stream(stream)))
    return logdet, sign, status


def logdet(models, x, opt=None, model_idx=None, x_off=None, n_items=None, stream=None, ws=None):
    """Single-spin log|det(1 + B_L...B_1)|, sign and status per item (SM Eq. S2).
    x: float64 GPU tensor [items, Ltau, N] (one model) or packed 1-D with x_off."""
    return _fermion(models, x, opt, model_idx, x_off, None, n_items, False, None, stream, ws)


def green(models, x, opt=None, model_idx=None, x_off=None, g_off=None, n_items=None, G=None,
          stream=None, ws=None):
    """As logdet, plus G = (1 + B_L...B_1)^{-1} (SM Eq. S3), G[i][j] = <c_i c_j^+>."""
    return _fermion(models, x, opt, model_idx, x_off, g_off, n_items, True, G, stream, ws)


def _chains(m, x, name="x"):
    if x.dim() != 3:
        raise ValueError("%s must be [chains, Ltau, N]" % name)
    _shape(x, (x.shape[0],) + _dims(m), name)
    return x.shape[0]


def eff_energy(m, eff, x, stream=None):
    torch = _torch()
    n = _chains(m, x)
    e = torch.empty(n, dtype=torch.float64, device=x.device)
    _abi.check(_abi.lib().slmc_eff_energy(C.byref(m), C.byref(eff), n, _dev_f64(x, "x"),
                                          C.c_void_p(e.data_ptr()), _stream(stream)))
    return e


def eff_sweep(m, eff, x, n_sweeps, seed, proposal_idx, stream=None):
    """n_sweeps checkerboard Metropolis sweeps of every chain of x [chains, Ltau, N], in
    place; returns the accepted-move count per chain."""
    torch = _torch()
    n = _chains(m, x)
    nacc = torch.empty(n, dtype=torch.int64, device=x.device)
    _abi.check(_abi.lib().slmc_eff_sweep(C.byref(m), C.byref(eff), n, _dev_f64(x, "x"),
                                         int(n_sweeps), C.c_uint64(seed), C.c_uint64(proposal_idx),
                                         C.c_void_p(nacc.data_ptr()), _stream(stream)))
    return nacc


def green_slices(m, x, n_wrap, opt=None, want_g=False, stream=None, ws=None):
    """G after every time slice (SM Eq. S3) and the CDW estimators per slice for the
    fields x [items, Ltau, N]: returns (s_nn [items, Ltau], m_st [items, Ltau], status
    [items], G_all [items, Ltau, N, N] or None)."""
    torch = _torch()
    n = _chains(m, x)
    opt = opt or options()
    L = _abi.lib()
    N, Lt = m.Lx * m.Ly, m.Ltau
    need = L.slmc_slices_workspace_bytes(C.byref(m), n, C.byref(opt))
    wsp, wsn = _ws_args(ws if ws is not None else _workspace(need, x.device, stream))
    s_nn = torch.empty((n, Lt), dtype=torch.float64, device=x.device)
    m_st = torch.empty((n, Lt), dtype=torch.float64, device=x.device)
    st = torch.empty(n, dtype=torch.int32, device=x.device)
    G = torch.empty((n, Lt, N, N), dtype=torch.float64, device=x.device) if want_g else None
    vp = C.c_void_p
    _abi.check(L.slmc_green_slices(C.byref(m), C.byref(opt), n, _dev_f64(x, "x"), int(n_wrap),
                                   None if G is None else vp(G.data_ptr()), vp(s_nn.data_ptr()),
                                   vp(m_st.data_ptr()), vp(st.data_ptr()), wsp, wsn, _stream(stream)))
    return s_nn, m_st, st, G


def dqmc_sweep(m, x, delta, n_rec, seed, sweep_idx, opt=None, want_g=False, stream=None, ws=None):
    """One DQMC local sweep of every chain of x [chains, Ltau, N], in place (SM Sec. I).
    Returns (accepted moves [chains] int64, status [chains] int32, G of the final fields
    [chains, N, N] or None)."""
    torch = _torch()
    n = _chains(m, x)
    opt = opt or options()
    L = _abi.lib()
    N = m.Lx * m.Ly
    need = L.slmc_dqmc_workspace_bytes(C.byref(m), n, C.byref(opt))
    wsp, wsn = _ws_args(ws if ws is not None else _workspace(need, x.device, stream))
    nacc = torch.empty(n, dtype=torch.int64, device=x.device)
    st = torch.empty(n, dtype=torch.int32, device=x.device)
    G = torch.empty((n, N, N), dtype=torch.float64, device=x.device) if want_g else None
    vp = C.c_void_p
    _abi.check(L.slmc_dqmc_sweep(C.byref(m), C.byref(opt), n, _dev_f64(x, "x"), float(delta), int(n_rec),
                                 C.c_uint64(seed), C.c_uint64(sweep_idx), vp(nacc.data_ptr()),
                                 None if G is None else vp(G.data_ptr()), vp(st.data_ptr()), wsp, wsn,
                                 _stream(stream)))
    return nacc, st, G


def dqmc_block(m, x, logw, n_updates, seed, sweep_idx, opt=None, stream=None, ws=None):
    """n_updates column-reflection block updates of every chain (SM Sec. I), in place;
    logw [chains] (cached log weight) is updated on accept.  Returns (accepted [chains]
    int64, status [chains] int32)."""
    torch = _torch()
    n = _chains(m, x)
    _shape(logw, (n,), "logw")
    opt = opt or options()
    L = _abi.lib()
    need = L.slmc_dqmc_workspace_bytes(C.byref(m), n, C.byref(opt))
    wsp, wsn = _ws_args(ws if ws is not None else _workspace(need, x.device, stream))
    nacc = torch.empty(n, dtype=torch.int64, device=x.device)
    st = torch.empty(n, dtype=torch.int32, device=x.device)
    vp = C.c_void_p
    _abi.check(L.slmc_dqmc_block(C.byref(m), C.byref(opt), n, _dev_f64(x, "x"), _dev_f64(logw, "logw"),
                                 int(n_updates), C.c_uint64(seed), C.c_uint64(sweep_idx),
                                 vp(nacc.data_ptr()), vp(st.data_ptr()), wsp, wsn, _stream(stream)))
    return nacc, st


TERMS = ("Jk", "J2", "Jp", "Jp6", "Js0", "Js1", "Js2", "Jt")


def eff_fit(m, x, logw, terms=("Jk", "Jp", "Jp6", "Js0", "Jt"), a=None, stream=None):
    """Least-squares fit of ln w ~ E0 - E_eff over the configurations x [n, Ltau, N]
    (Eq. 5): returns (coef [9] = (E0, J in TERMS order), features [n, 8]).  a defaults to
    the well position lambda / omega0^2."""
    torch = _torch()
    n = _chains(m, x)
    _shape(logw, (n,), "logw")
    mask = 0
    for t in terms:
        mask |= 1 << TERMS.index(t)
    a = m.lam / m.omega0 ** 2 if a is None else float(a)
    L = _abi.lib()
    ws = _workspace(L.slmc_fit_workspace_bytes(n), x.device, stream)
    wsp, wsn = _ws_args(ws)
    coef = torch.empty(9, dtype=torch.float64, device=x.device)
    F = torch.empty((n, 8), dtype=torch.float64, device=x.device)
    vp = C.c_void_p
    _abi.check(L.slmc_eff_fit(C.byref(m), a, n, _dev_f64(x, "x"), _dev_f64(logw, "logw"), mask,
                              vp(F.data_ptr()), vp(coef.data_ptr()), wsp, wsn, _stream(stream)))
    return coef, F


def step(m, eff, x_cur, x_prop, logw_cur, eeff_cur, n_sweeps, n_clusters, seed, counter, opt=None,
         G_prop=None, out=None, stream=None, ws=None):
    """One whole SLMC step (slmc_step): proposal from x_cur into x_prop, accept into x_cur,
    logw_cur, eeff_cur; the proposal index is read from the device tensor counter (uint64
    stored as int64, shape [1]) and incremented.  out: optional dict of preallocated output
    tensors (accepted, log_ratio, status, n_local) -- pass it when capturing into a graph.
    Returns that dict."""
    torch = _torch()
    n = _chains(m, x_cur, "x_cur")
    _shape(x_prop, tuple(x_cur.shape), "x_prop")
    _shape(logw_cur, (n,), "logw_cur")
    _shape(eeff_cur, (n,), "eeff_cur")
    if counter.dtype != torch.int64 or counter.numel() != 1 or not counter.is_cuda:
        raise ValueError("counter must be a one-element int64 GPU tensor")
    if G_prop is not None:
        N = m.Lx * m.Ly
        _shape(G_prop, (n, N, N), "G_prop")
    opt = opt or options()
    L = _abi.lib()
    need = L.slmc_accept_workspace_bytes(C.byref(m), n, C.byref(opt))
    wsp, wsn = _ws_args(ws if ws is not None else _workspace(need, x_cur.device, stream))
    if out is None:
        out = {"accepted": torch.empty(n, dtype=torch.uint8, device=x_cur.device),
               "log_ratio": torch.empty(n, dtype=torch.float64, device=x_cur.device),
               "status": torch.empty(n, dtype=torch.int32, device=x_cur.device),
               "n_local": torch.empty(n, dtype=torch.int64, device=x_cur.device)}
    vp = C.c_void_p
    _abi.check(L.slmc_step(C.byref(m), C.byref(eff), C.byref(opt), n, _dev_f64(x_cur, "x_cur"),
                           _dev_f64(x_prop, "x_prop"), _dev_f64(logw_cur, "logw_cur"),
                           _dev_f64(eeff_cur, "eeff_cur"), int(n_sweeps), int(n_clusters),
                           C.c_uint64(seed), vp(counter.data_ptr()), vp(out["accepted"].data_ptr()),
                           vp(out["log_ratio"].data_ptr()),
                           None if G_prop is None else _dev_f64(G_prop, "G_prop"),
                           vp(out["status"].data_ptr()), vp(out["n_local"].data_ptr()), wsp, wsn,
                           _stream(stream)))
    return out


SCHEDULES = {0: "default", 1: "eager", 2: "gated", 3: "serial", 4: "gated, V behind segments"}


def _tuning_dict(t):
    return {"schedule": SCHEDULES.get(t.schedule, t.schedule), "seg_ahead": t.seg_ahead, "gate": t.gate,
            "seg_mode": t.seg_mode, "seg_cb": t.seg_cb, "ms_per_call": round(t.ms_per_call, 4)}


def autotune(m, x, opt=None, stream=None):
    """Runs the library's autotuner on the fields x [items, Ltau, N] (slmc_autotune): the
    fastest bitwise-equal schedule and tile choice for this model, precision and batch size
    is kept for later calls.  Returns (choice dict, candidates tried, rejected)."""
    torch = _torch()
    n = _chains(m, x)
    opt = opt or options()
    L = _abi.lib()
    need = L.slmc_workspace_bytes(C.byref(m), 1, C.byref(_BatchArgs(n).batch), C.byref(opt)) + \
        6 * ((8 * n + 255) // 256 * 256)
    wsp, wsn = _ws_args(_workspace(need, x.device, stream))
    t = _abi.Tuning()
    tried, rej = C.c_int32(), C.c_int32()
    _abi.check(L.slmc_autotune(C.byref(m), C.byref(opt), n, _dev_f64(x, "x"), wsp, wsn, _stream(stream),
                               C.byref(t), C.byref(tried), C.byref(rej)))
    return _tuning_dict(t), tried.value, rej.value


def tuning(m, n_items, opt=None):
    """(choice dict, tuned?) in effect for this model, precision and batch size."""
    opt = opt or options()
    t = _abi.Tuning()
    tuned = C.c_int32()
    _abi.check(_abi.lib().slmc_tuning_lookup(C.byref(m), C.byref(opt), int(n_items), C.byref(t),
                                             C.byref(tuned)))
    return _tuning_dict(t), bool(tuned.value)


def eff_wolff(m, eff, x, n_clusters, seed, proposal_idx, stream=None):
    """n_clusters modified Wolff cluster moves of every chain of x [chains, Ltau, N], in
    place (SM Sec. IV); returns the cluster sizes [chains, n_clusters]."""
    torch = _torch()
    n = _chains(m, x)
    sizes = torch.empty((n, max(int(n_clusters), 0)), dtype=torch.int32, device=x.device)
    _abi.check(_abi.lib().slmc_eff_wolff(C.byref(m), C.byref(eff), n, _dev_f64(x, "x"),
                                         int(n_clusters), C.c_uint64(seed), C.c_uint64(proposal_idx),
                                         C.c_void_p(sizes.data_ptr()), _stream(stream)))
    return sizes


def eff_propose(m, eff, x, n_sweeps, n_clusters, seed, proposal_idx, stream=None):
    """The cumulative proposal of every chain of x [chains, Ltau, N], in place: sweeps and
    cluster moves in the order of the proposal's coin.  Returns (accepted local moves
    [chains] int64, cluster sizes [chains, n_clusters] int32)."""
    torch = _torch()
    n = _chains(m, x)
    nacc = torch.empty(n, dtype=torch.int64, device=x.device)
    sizes = torch.empty((n, max(int(n_clusters), 0)), dtype=torch.int32, device=x.device)
    _abi.check(_abi.lib().slmc_eff_propose(C.byref(m), C.byref(eff), n, _dev_f64(x, "x"),
                                           int(n_sweeps), int(n_clusters), C.c_uint64(seed),
                                           C.c_uint64(proposal_idx), C.c_void_p(nacc.data_ptr()),
                                           C.c_void_p(sizes.data_ptr()), _stream(stream)))
    return nacc, sizes


def log_weight(m, x, opt=None, stream=None, ws=None):
    """log w = -dtau S_Bose + 2 log|det M| per chain of x [chains, Ltau, N].  Returns
    (logw, status): status[c] != 0 marks a chain whose log-det failed (logw NaN)."""
    torch = _torch()
    n = _chains(m, x)
    opt = opt or options()
    L = _abi.lib()
    need = L.slmc_accept_workspace_bytes(C.byref(m), n, C.byref(opt))
    wsp, wsn = _ws_args(ws if ws is not None else _workspace(need, x.device, stream))
    lw = torch.empty(n, dtype=torch.float64, device=x.device)
    st = torch.empty(n, dtype=torch.int32, device=x.device)
    _abi.check(L.slmc_log_weight(C.byref(m), C.byref(opt), n, _dev_f64(x, "x"),
                                 C.c_void_p(lw.data_ptr()), C.c_void_p(st.data_ptr()), wsp, wsn,
                                 _stream(stream)))
    return lw, st


def cumulative_accept(m, eff, x_cur, x_prop, logw_cur, eeff_cur, seed, proposal_idx, opt=None,
                      stream=None, ws=None, G_prop=None):
    """Eq. 6 for one proposal per chain; x_cur, logw_cur, eeff_cur are updated in place on
    accept.  G_prop (optional, [chains, N, N]) receives the proposals' Green's functions.
    Returns (accepted uint8, log_ratio float64, status int32): a proposal whose log-det
    failed (status != 0) has log_ratio NaN and is rejected."""
    torch = _torch()
    opt = opt or options()
    L = _abi.lib()
    n = _chains(m, x_cur, "x_cur")
    _shape(x_prop, tuple(x_cur.shape), "x_prop")
    _shape(logw_cur, (n,), "logw_cur")
    _shape(eeff_cur, (n,), "eeff_cur")
    if G_prop is not None:
        N = m.Lx * m.Ly
        _shape(G_prop, (n, N, N), "G_prop")
    need = L.slmc_accept_workspace_bytes(C.byref(m), n, C.byref(opt))
    wsp, wsn = _ws_args(ws if ws is not None else _workspace(need, x_cur.device, stream))
    acc = torch.empty(n, dtype=torch.uint8, device=x_cur.device)
    lr = torch.empty(n, dtype=torch.float64, device=x_cur.device)
    st = torch.empty(n, dtype=torch.int32, device=x_cur.device)
    vp = C.c_void_p
    _abi.check(L.slmc_cumulative_accept(
        C.byref(m), C.byref(eff), C.byref(opt), n, _dev_f64(x_cur, "x_cur"),
        _dev_f64(x_prop, "x_prop"), _dev_f64(logw_cur, "logw_cur"), _dev_f64(eeff_cur, "eeff_cur"),
        C.c_uint64(seed), C.c_uint64(proposal_idx), vp(acc.data_ptr()), vp(lr.data_ptr()),
        None if G_prop is None else _dev_f64(G_prop, "G_prop"), vp(st.data_ptr()), wsp, wsn,
        _stream(stream)))
    return acc, lr, st


def green_noalloc(m, x, opt=None, want_g=True, G=None, stream=None):
    """slmc_green_noalloc: log-det, sign, (G) and status of the fields x [items, Ltau, N] of
    one model, with the library's static scratch as workspace (no device allocation in the
    library; the outputs are allocated here unless G is passed)."""
    torch = _torch()
    n = _chains(m, x)
    N = m.Lx * m.Ly
    if G is not None:
        _shape(G, (n, N, N), "G")
    xp = _dev_f64(x, "x")
    opt = opt or options()
    logdet = torch.empty(n, dtype=torch.float64, device=x.device)
    sign = torch.empty(n, dtype=torch.int8, device=x.device)
    status = torch.empty(n, dtype=torch.int32, device=x.device)
    if want_g and G is None:
        G = torch.empty((n, N, N), dtype=torch.float64, device=x.device)
    vp = C.c_void_p
    _abi.check(_abi.lib().slmc_green_noalloc(
        C.byref(m), C.byref(opt), n, xp, vp(logdet.data_ptr()), vp(sign.data_ptr()),
        _dev_f64(G, "G") if want_g else None, vp(status.data_ptr()), _stream(stream)))
    return (logdet, sign, G, status) if want_g else (logdet, sign, status)
