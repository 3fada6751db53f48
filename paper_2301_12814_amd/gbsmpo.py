"""Thin ctypes binding of libgbsmpo.so (argument marshalling only).

Every step of the simulation runs in the HIP kernels of the library; this
module only converts Python/NumPy arguments to the C ABI declared in
``include/gbs_mpo.h``.  There is no fallback: if the library is missing or
fails to load, an error is raised.
"""
from __future__ import annotations

import ctypes
import os

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
# GBSMPO_LIB overrides the in-tree library (variant builds of the same sources)
LIB_PATH = os.environ.get("GBSMPO_LIB") or os.path.join(_HERE, "libgbsmpo.so")

MPO_OK, MPO_EINVAL, MPO_ENOMEM, MPO_EDEVICE, MPO_ENUMERIC, MPO_EBUSY = 0, -1, -2, -3, -4, -5
MPO_FP64, MPO_MIXED = 0, 1

_lib = None


class GbsMpoError(RuntimeError):
    def __init__(self, code: int, msg: str):
        super().__init__(f"[{code}] {msg}")
        self.code = code


def lib() -> ctypes.CDLL:
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise GbsMpoError(MPO_EDEVICE, f"{LIB_PATH} not built (run __graft_entry__.build())")
        L = ctypes.CDLL(LIB_PATH)
        c_int, c_double, c_void_p = ctypes.c_int, ctypes.c_double, ctypes.c_void_p
        pd = ctypes.POINTER(ctypes.c_double)
        pi = ctypes.POINTER(ctypes.c_int)
        pll = ctypes.POINTER(ctypes.c_longlong)
        L.mpo_init_lossy_squeezed.argtypes = [c_int, pd, c_double, c_int, c_int, c_int, c_void_p,
                                              ctypes.POINTER(c_void_p)]
        L.mpo_init_lossy_squeezed_total_cap.argtypes = L.mpo_init_lossy_squeezed.argtypes
        L.mpo_apply_bs_layer.argtypes = [c_void_p, c_int, pi, pd, pd]
        L.mpo_apply_phases.argtypes = [c_void_p, pd]
        L.mpo_entropy.argtypes = [c_void_p, pd, pd]
        L.mpo_photon_marginals.argtypes = [c_void_p, pd, pd]
        L.mpo_photon_marginals_noalloc.argtypes = [c_void_p, pd, pd]
        L.mpo_renyi.argtypes = [c_void_p, c_double, pd]
        L.gbs_asymptotic_ee.argtypes = [c_double, c_double, c_int, c_double, c_int, c_double,
                                        pd, pd]
        L.gbs_run_until_saturation.argtypes = [c_int, pd, c_double, c_int, c_int, c_int, pd, c_int,
                                               pi, pd, pi, pd]
        L.gbs_chi_search.argtypes = [c_int, pd, c_double, c_int, c_int, pd, c_int, c_int, c_double,
                                     c_int, pi, pd, c_int, pi, pi, pd]
        L.mpo_sync.argtypes = [c_void_p]
        L.mpo_get_bond.argtypes = [c_void_p, c_int, pi, pd, pi]
        L.mpo_get_site.argtypes = [c_void_p, c_int, pd]
        L.mpo_layer_stats.argtypes = [c_void_p, pll]
        L.mpo_free.argtypes = [c_void_p]
        L.mpo_free.restype = None
        L.mpo_last_error.restype = ctypes.c_char_p
        L.gbs_clements_decompose.argtypes = [c_int, pd, pi, pi, pd, pd, pd]
        L.mpo_set_profiling.argtypes = [c_void_p, c_int]
        L.mpo_get_profile.argtypes = [c_void_p, pd, pll, pd]
        L.mpo_layer_blocks.argtypes = [c_void_p, c_int, pi]
        L.mpo_get_contraction_work.argtypes = [c_void_p, pd]
        L.gbs_device_memory.argtypes = [pll, pll]
        L.gbs_device_memory.restype = c_int
        L.gbs_set_svd_route.argtypes = [c_int, c_int]
        L.gbs_set_svd_route.restype = c_int
        pe = ctypes.POINTER(c_void_p)
        L.mpo_engine_projected_bytes.argtypes = [c_int, c_int, c_int]
        L.mpo_engine_projected_bytes.restype = ctypes.c_longlong
        L.mpo_engine_create.argtypes = [c_void_p, c_int, ctypes.c_longlong, pe]
        L.mpo_engine_free.argtypes = [c_void_p]
        L.mpo_engine_free.restype = None
        L.mpo_engine_add.argtypes = [c_void_p, c_int, pd, c_double, c_int, c_int, pd, pi]
        L.mpo_engine_step.argtypes = [c_void_p, pi]
        L.mpo_engine_result.argtypes = [c_void_p, c_int, pi, pd, pd, pd]
        L.mpo_engine_release.argtypes = [c_void_p, c_int]
        L.mpo_engine_set_sweep_limit.argtypes = [c_void_p, c_int, c_int]
        L.mpo_engine_set_profiling.argtypes = [c_void_p, c_int]
        L.mpo_engine_get_profile.argtypes = [c_void_p, pd, pll, pd]
        for name in ("mpo_engine_create", "mpo_engine_add", "mpo_engine_step",
                     "mpo_engine_result", "mpo_engine_release", "mpo_engine_set_sweep_limit",
                     "mpo_engine_set_profiling",
                     "mpo_engine_get_profile"):
            getattr(L, name).restype = c_int
        for name in ("mpo_layer_blocks", "mpo_set_profiling", "mpo_get_profile", "mpo_init_lossy_squeezed",
                     "mpo_init_lossy_squeezed_total_cap", "mpo_apply_bs_layer", "mpo_apply_phases",
                     "mpo_entropy", "mpo_photon_marginals", "mpo_photon_marginals_noalloc",
                     "mpo_sync", "mpo_get_bond", "mpo_renyi", "gbs_asymptotic_ee",
                     "gbs_run_until_saturation", "gbs_chi_search", "mpo_get_contraction_work",
                     "mpo_get_site", "mpo_layer_stats", "gbs_clements_decompose"):
            getattr(L, name).restype = c_int
        _lib = L
    return _lib


def _check(rc: int):
    if rc < 0:
        raise GbsMpoError(rc, lib().mpo_last_error().decode())
    return rc


def _dp(a):
    return a.ctypes.data_as(ctypes.POINTER(ctypes.c_double))


def _ip(a):
    return a.ctypes.data_as(ctypes.POINTER(ctypes.c_int))


def _stream_handle(stream):
    """A raw hipStream_t (int) of the system HIP runtime the library links, or
    None for the library's own stream.  (PyTorch wheels bundle a second HIP
    runtime whose streams are not valid here.)"""
    if stream is None:
        return None
    if isinstance(stream, int):
        return ctypes.c_void_p(stream)
    raise TypeError("stream must be None or an int hipStream_t of the library's HIP runtime")


def clements(U: np.ndarray):
    """Library Clements decomposition: (layers, phases); each layer is a tuple of
    arrays (left_site int32, theta, phi) in application order."""
    U = np.ascontiguousarray(U, dtype=complex)
    M = U.shape[0]
    G = M * (M - 1) // 2
    ure = np.ascontiguousarray(np.stack([U.real, U.imag], axis=-1).reshape(-1))
    ptr = np.zeros(M + 1, dtype=np.int32)
    site = np.zeros(max(G, 1), dtype=np.int32)
    th = np.zeros(max(G, 1))
    ph = np.zeros(max(G, 1))
    phase = np.zeros(M)
    nl = _check(lib().gbs_clements_decompose(M, _dp(ure), _ip(ptr), _ip(site), _dp(th), _dp(ph),
                                             _dp(phase)))
    layers = [(site[ptr[l]:ptr[l + 1]].copy(), th[ptr[l]:ptr[l + 1]].copy(),
               ph[ptr[l]:ptr[l + 1]].copy()) for l in range(nl)]
    return layers, phase


class MPO:
    """One simulation: lossy squeezed product state evolved by beam-splitter layers."""

    def __init__(self, M, r, eta, d, chi, precision=MPO_FP64, stream=None, total_cap=False):
        """total_cap: d bounds the total photon number (mpo_init_lossy_squeezed_total_cap)."""
        L = lib()
        r = np.ascontiguousarray(np.broadcast_to(np.asarray(r, dtype=float), (M,)))
        h = ctypes.c_void_p()
        init = L.mpo_init_lossy_squeezed_total_cap if total_cap else L.mpo_init_lossy_squeezed
        _check(init(int(M), _dp(r), float(eta), int(d), int(chi), int(precision),
                    _stream_handle(stream), ctypes.byref(h)))
        self._h = h
        self.M, self.d, self.chi = int(M), int(d), int(chi)

    def close(self):
        if getattr(self, "_h", None) is not None and self._h.value:
            lib().mpo_free(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def __enter__(self):
        return self

    def __exit__(self, *exc):
        self.close()

    def apply_layer(self, sites, theta, phi):
        sites = np.ascontiguousarray(sites, dtype=np.int32)
        theta = np.ascontiguousarray(theta, dtype=float)
        phi = np.ascontiguousarray(phi, dtype=float)
        _check(lib().mpo_apply_bs_layer(self._h, len(sites), _ip(sites), _dp(theta), _dp(phi)))

    def apply_phases(self, phase):
        phase = np.ascontiguousarray(phase, dtype=float)
        _check(lib().mpo_apply_phases(self._h, _dp(phase)))

    def entropy(self):
        S = np.zeros(max(self.M - 1, 1))
        smax = ctypes.c_double()
        _check(lib().mpo_entropy(self._h, _dp(S), ctypes.byref(smax)))
        return S[: self.M - 1], smax.value

    def marginals(self):
        P = np.zeros(self.M * self.d)
        tr = ctypes.c_double()
        _check(lib().mpo_photon_marginals(self._h, _dp(P), ctypes.byref(tr)))
        return P.reshape(self.M, self.d), tr.value

    def renyi(self, alpha):
        """Renyi-alpha operator entropies of bonds 1..M-1 (bits)."""
        S = np.zeros(max(self.M - 1, 1))
        _check(lib().mpo_renyi(self._h, float(alpha), _dp(S)))
        return S[: self.M - 1]

    def marginals_noalloc(self):
        """mpo_photon_marginals_noalloc: the marginals from the library's static
        scratch array (no device allocation)."""
        P = np.zeros(self.M * self.d)
        tr = ctypes.c_double()
        _check(lib().mpo_photon_marginals_noalloc(self._h, _dp(P), ctypes.byref(tr)))
        return P.reshape(self.M, self.d), tr.value

    def bond(self, b):
        D = ctypes.c_int()
        lam = np.zeros(self.chi)
        ch = np.zeros(2 * self.chi, dtype=np.int32)
        _check(lib().mpo_get_bond(self._h, int(b), ctypes.byref(D), _dp(lam), _ip(ch)))
        n = D.value
        return lam[:n].copy(), ch[: 2 * n].reshape(n, 2).copy()

    def site(self, j):
        G = np.zeros(2 * self.chi * self.chi)
        _check(lib().mpo_get_site(self._h, int(j), _dp(G)))
        Dl = self.bond(j)[0].shape[0]
        Dr = self.bond(j + 1)[0].shape[0]
        return (G[0::2] + 1j * G[1::2])[: Dl * Dr].reshape(Dl, Dr)

    def layer_stats(self):
        s = (ctypes.c_longlong * 6)()
        _check(lib().mpo_layer_stats(self._h, s))
        keys = ("blocks", "elements", "candidates", "max_rows", "max_cols", "max_sweeps")
        return dict(zip(keys, list(s)))

    def sync(self):
        _check(lib().mpo_sync(self._h))

    def contraction_flops(self):
        """Algorithmic Theta-contraction flops since profiling was enabled."""
        f = ctypes.c_double()
        _check(lib().mpo_get_contraction_work(self._h, ctypes.byref(f)))
        return f.value

    def layer_blocks(self):
        """Sector histogram of the last layer: int array [nblocks, 8] with
        (gate, n, n', rows, cols, computed, sweeps, kept)."""
        n = _check(lib().mpo_layer_blocks(self._h, 0, None))
        out = np.zeros(8 * max(n, 1), dtype=np.int32)
        _check(lib().mpo_layer_blocks(self._h, n, _ip(out)))
        return out[: 8 * n].reshape(n, 8)

    PHASES = ("fock", "plan", "contract", "svd", "select", "scatter", "entropy", "unused")

    def set_profiling(self, on: bool = True):
        _check(lib().mpo_set_profiling(self._h, 1 if on else 0))

    def profile(self):
        """(per-phase summed ms, per-phase timed layers, work dict)."""
        ms = np.zeros(8)
        n = np.zeros(8, dtype=np.int64)
        work = np.zeros(4)
        _check(lib().mpo_get_profile(self._h, _dp(ms),
                                     n.ctypes.data_as(ctypes.POINTER(ctypes.c_longlong)),
                                     _dp(work)))
        return (dict(zip(self.PHASES, ms.tolist())), dict(zip(self.PHASES, n.tolist())),
                dict(svd_flops=work[0], elements=work[1], candidates=work[2], layers=work[3]))


def asymptotic_ee(r, mu, n_max, n_inputs, alpha=1.0, theta=np.pi / 4):
    """App. C single-mode estimate of the operator EE (or Renyi-alpha entropy)
    times n_inputs; returns (S, normalised spectrum)."""
    S = ctypes.c_double()
    spec = np.zeros((int(n_max) + 1) ** 2)
    _check(lib().gbs_asymptotic_ee(float(r), float(mu), int(n_max), float(theta), int(n_inputs),
                                   float(alpha), ctypes.byref(S), _dp(spec)))
    return S.value, spec


def _ure(U):
    U = np.ascontiguousarray(U, dtype=complex)
    return np.ascontiguousarray(np.stack([U.real, U.imag], axis=-1).reshape(-1))


def run_until_saturation(M, r, eta, d, chi, U, patience=10, precision=MPO_FP64):
    """App. A stop rule; returns (layers_used, S_max, layer_of_max, trace)."""
    r = np.ascontiguousarray(np.broadcast_to(np.asarray(r, dtype=float), (M,)))
    ure = _ure(U)
    used, at = ctypes.c_int(), ctypes.c_int()
    smax, tr = ctypes.c_double(), ctypes.c_double()
    _check(lib().gbs_run_until_saturation(int(M), _dp(r), float(eta), int(d), int(chi),
                                          int(precision), _dp(ure), int(patience),
                                          ctypes.byref(used), ctypes.byref(smax),
                                          ctypes.byref(at), ctypes.byref(tr)))
    return used.value, smax.value, at.value, tr.value


def chi_search(M, r, eta, d, U, chi0, chi_max, target, refine, precision=MPO_FP64,
               max_trials=64):
    """App. A bond-dimension search; returns (chi_found, error, [(chi, error)])."""
    r = np.ascontiguousarray(np.broadcast_to(np.asarray(r, dtype=float), (M,)))
    ure = _ure(U)
    cf, ef, nt = ctypes.c_int(), ctypes.c_double(), ctypes.c_int()
    tc = np.zeros(max_trials, dtype=np.int32)
    te = np.zeros(max_trials)
    _check(lib().gbs_chi_search(int(M), _dp(r), float(eta), int(d), int(precision), _dp(ure),
                                int(chi0), int(chi_max), float(target), int(refine),
                                ctypes.byref(cf), ctypes.byref(ef), int(max_trials),
                                ctypes.byref(nt), _ip(tc), _dp(te)))
    n = min(nt.value, max_trials)
    return cf.value, ef.value, list(zip(tc[:n].tolist(), te[:n].tolist()))


def device_memory():
    """(free, total) device bytes of the current device."""
    f, t = ctypes.c_longlong(), ctypes.c_longlong()
    _check(lib().gbs_device_memory(ctypes.byref(f), ctypes.byref(t)))
    return f.value, t.value


def set_svd_route(lds_limit_bytes=0, qr_enable=True):
    """Routing of the block SVDs (LDS budget, QR reduction); 0 = device budget."""
    _check(lib().gbs_set_svd_route(int(lds_limit_bytes), 1 if qr_enable else 0))


def projected_bytes(M, d, chi) -> int:
    """Device bytes a simulation is admitted against (state + its workspace share)."""
    return int(lib().mpo_engine_projected_bytes(int(M), int(d), int(chi)))


class Engine:
    """Continuous-batching engine: every step applies the next beam-splitter
    layer of every running simulation in one batched launch sequence."""

    def __init__(self, precision=MPO_FP64, budget_bytes=0, stream=None):
        h = ctypes.c_void_p()
        _check(lib().mpo_engine_create(_stream_handle(stream), int(precision),
                                       int(budget_bytes), ctypes.byref(h)))
        self._h = h
        self.meta = {}

    def close(self):
        if getattr(self, "_h", None) is not None and self._h.value:
            lib().mpo_engine_free(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def __enter__(self):
        return self

    def __exit__(self, *exc):
        self.close()

    def add(self, M, r, eta, d, chi, U):
        """Admit a simulation (raises GbsMpoError MPO_ENOMEM if it does not fit)."""
        r = np.ascontiguousarray(np.broadcast_to(np.asarray(r, dtype=float), (M,)))
        U = np.ascontiguousarray(U, dtype=complex)
        ure = np.ascontiguousarray(np.stack([U.real, U.imag], axis=-1).reshape(-1))
        sid = ctypes.c_int()
        _check(lib().mpo_engine_add(self._h, int(M), _dp(r), float(eta), int(d), int(chi),
                                    _dp(ure), ctypes.byref(sid)))
        self.meta[sid.value] = (int(M), int(d))
        return sid.value

    def step(self):
        n = ctypes.c_int()
        _check(lib().mpo_engine_step(self._h, ctypes.byref(n)))
        return n.value

    def result(self, sid):
        """None while running, else dict(S_max, trace, P)."""
        M, d = self.meta[sid]
        done = ctypes.c_int()
        smax = ctypes.c_double()
        tr = ctypes.c_double()
        P = np.zeros(M * d)
        _check(lib().mpo_engine_result(self._h, int(sid), ctypes.byref(done), ctypes.byref(smax),
                                       ctypes.byref(tr), _dp(P)))
        if not done.value:
            return None
        return {"S_max": smax.value, "trace": tr.value, "P": P.reshape(M, d)}

    def release(self, sid):
        _check(lib().mpo_engine_release(self._h, int(sid)))
        self.meta.pop(sid, None)

    def set_sweep_limit(self, sid, max_sweeps):
        """Failure injection: Jacobi sweep limit of one running simulation."""
        _check(lib().mpo_engine_set_sweep_limit(self._h, int(sid), int(max_sweeps)))

    def set_profiling(self, on=True):
        _check(lib().mpo_engine_set_profiling(self._h, 1 if on else 0))

    def profile(self):
        ms = np.zeros(8)
        n = np.zeros(8, dtype=np.int64)
        work = np.zeros(4)
        _check(lib().mpo_engine_get_profile(self._h, _dp(ms),
                                            n.ctypes.data_as(ctypes.POINTER(ctypes.c_longlong)),
                                            _dp(work)))
        return (dict(zip(MPO.PHASES, ms.tolist())), dict(zip(MPO.PHASES, n.tolist())),
                dict(svd_flops=work[0], elements=work[1], candidates=work[2], layers=work[3]))
