"""MI355X (gfx950) Ising hot path for uplink ML-MIMO detection and downlink
vector-perturbation precoding (after "MMGaP", arXiv 2510.01579).

This module is a thin ctypes binding of the C ABI in include/mmgap.h
(libmmgap.so, built in-tree by ``paper_2510_01579_amd.build``).  It marshals
torch tensors (device memory) and the current HIP stream; every step of the
computation runs in the library's HIP kernels.  There is no CPU fallback: if
the library is missing or no GPU is present the calls raise.

Entry points (same names as the C ABI, without the ``mmgap_`` prefix):
``build_ising``, ``solve``, ``detect``, ``detect_delta``, ``detect_sic``,
``detect_e``, ``vpp_precode``; ``Context`` owns a
library context (device, scratch, HBM budget); ``Context.plan_create`` returns a
``Plan`` (``plan_launch``, ``plan_info``, ``plan_destroy``) that runs a batch of
mixed jobs in one persistent launch; ``Context.server_start`` runs the native
serving loop (``server_submit``, ``server_poll``, ``server_drain``,
``server_stop``) that admits jobs as they arrive.
"""
from __future__ import annotations

import ctypes
import math
import os
import threading

import numpy as np

_PKG = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_PKG, "libmmgap.so")

KIND_DET = 0
KIND_VPP = 1

STATUS = {0: "MMGAP_OK", -1: "MMGAP_EINVAL", -2: "MMGAP_ENOMEM", -3: "MMGAP_EDEVICE",
          -4: "MMGAP_EUNSUPPORTED", -5: "MMGAP_EBUSY"}

EXPORTS = ("mmgap_create", "mmgap_destroy", "mmgap_last_error", "mmgap_build_ising",
           "mmgap_solve", "mmgap_detect", "mmgap_detect_delta", "mmgap_detect_sic",
           "mmgap_detect_e", "mmgap_cim_chains", "mmgap_vpp_precode",
           "mmgap_set_profiling", "mmgap_set_option",
           "mmgap_last_profile", "mmgap_plan_create", "mmgap_plan_launch", "mmgap_plan_info",
           "mmgap_plan_destroy", "mmgap_server_start", "mmgap_server_submit",
           "mmgap_server_poll", "mmgap_server_stats", "mmgap_server_drain", "mmgap_server_stop")

PLAN_GRAPH = 1
PLAN_PERSISTENT = 2
OPT_STAGE_LAUNCHES = 1


class MmgapError(RuntimeError):
    def __init__(self, code: int, msg: str):
        super().__init__(f"{STATUS.get(code, code)}: {msg}")
        self.code = code


class Problem(ctypes.Structure):
    _fields_ = [("kind", ctypes.c_int), ("n_rx", ctypes.c_int), ("n_tx", ctypes.c_int),
                ("qam", ctypes.c_int), ("n_sc", ctypes.c_int), ("n_sym", ctypes.c_int),
                ("noise_var", ctypes.c_float), ("tau", ctypes.c_float)]


class CimParams(ctypes.Structure):
    """mmgap_cim_params: constants of the CIM-CAC model."""
    _fields_ = [("dt", ctypes.c_float), ("f_mvm", ctypes.c_int), ("p", ctypes.c_float),
                ("a", ctypes.c_float), ("zeta", ctypes.c_float), ("eps", ctypes.c_float),
                ("amp0", ctypes.c_float)]


class Schedule(ctypes.Structure):
    _fields_ = [("chains", ctypes.c_int), ("sweeps", ctypes.c_int),
                ("beta2", ctypes.POINTER(ctypes.c_float)), ("seed", ctypes.c_uint64),
                ("init", ctypes.c_int), ("dynamics", ctypes.c_int),
                ("cim", ctypes.POINTER(CimParams)), ("inst_base", ctypes.c_uint32)]


DYN_METROPOLIS, DYN_CIM = 0, 1
GUESS_MMSE, GUESS_SIC = 1, 2
# CIM-CAC constants used when a caller gives only some of them: the paper's
# integration step and coupling refresh period (dt = 0.02, f_mvm = 2; 128 steps
# cover its reference integration length 2.56); a, p, zeta, eps and the initial
# amplitude scale are this library's choice (the paper leaves them open).
CIM_DEFAULTS = dict(dt=0.02, f_mvm=2, p=0.9, a=1.0, zeta=1.0, eps=1.0, amp0=0.1)
CIM_STEPS = 128


class ServerStats(ctypes.Structure):
    """mmgap_server_stats_t."""
    _fields_ = [("completed", ctypes.c_ulonglong), ("missed", ctypes.c_ulonglong),
                ("p50_us", ctypes.c_double), ("p99_us", ctypes.c_double),
                ("max_us", ctypes.c_double)]


class Job(ctypes.Structure):
    _fields_ = [("prob", Problem), ("sched", Schedule), ("H", ctypes.c_void_p),
                ("y_or_u", ctypes.c_void_p), ("out0", ctypes.c_void_p),
                ("out1", ctypes.c_void_p), ("out2", ctypes.c_void_p), ("stages", ctypes.c_int),
                ("guesses", ctypes.c_int)]


_lib = None
_lib_lock = threading.Lock()


def lib() -> ctypes.CDLL:
    """Load libmmgap.so (raises if it has not been built)."""
    global _lib
    with _lib_lock:
        if _lib is None:
            if not os.path.exists(LIB_PATH):
                raise RuntimeError(f"{LIB_PATH} is missing: build it with "
                                   "`python -m paper_2510_01579_amd.build`")
            L = ctypes.CDLL(LIB_PATH)
            vp, i, f32 = ctypes.c_void_p, ctypes.c_int, ctypes.c_float
            L.mmgap_create.argtypes = [ctypes.POINTER(vp), i, ctypes.c_size_t]
            L.mmgap_destroy.argtypes = [vp]
            L.mmgap_last_error.argtypes = [vp]
            L.mmgap_last_error.restype = ctypes.c_char_p
            P = ctypes.POINTER(Problem)
            S = ctypes.POINTER(Schedule)
            L.mmgap_build_ising.argtypes = [vp, P, vp, vp, vp, vp, vp, vp, vp, vp, vp]
            L.mmgap_solve.argtypes = [vp, i, i, i, vp, vp, i, vp, vp, S, vp, vp, vp, vp]
            L.mmgap_detect.argtypes = [vp, P, vp, vp, S, vp, vp, vp]
            L.mmgap_detect_noalloc.argtypes = [vp, P, vp, vp, S, vp, vp, vp]
            L.mmgap_detect_delta.argtypes = [vp, P, vp, vp, S, i, vp, vp, vp, vp]
            L.mmgap_detect_sic.argtypes = [vp, P, vp, vp, vp, vp, vp, vp, vp]
            L.mmgap_detect_e.argtypes = [vp, P, vp, vp, S, i, i, vp, vp, vp, vp]
            L.mmgap_cim_chains.argtypes = [vp, i, i, i, vp, vp, i, vp, vp, S, vp, vp, vp, vp]
            L.mmgap_vpp_precode.argtypes = [vp, P, vp, vp, S, vp, vp, vp, vp]
            L.mmgap_set_profiling.argtypes = [vp, i]
            L.mmgap_set_option.argtypes = [vp, i, i]
            L.mmgap_last_profile.argtypes = [vp, ctypes.POINTER(f32), i]
            L.mmgap_plan_create.argtypes = [vp, i, ctypes.POINTER(Job), i, i, ctypes.POINTER(vp)]
            L.mmgap_plan_launch.argtypes = [vp, vp]
            L.mmgap_plan_info.argtypes = [vp, ctypes.POINTER(i), ctypes.POINTER(i)]
            L.mmgap_plan_destroy.argtypes = [vp]
            L.mmgap_server_start.argtypes = [vp, i, ctypes.c_size_t, i]
            L.mmgap_server_submit.argtypes = [vp, ctypes.POINTER(Job), vp,
                                              ctypes.POINTER(ctypes.c_ulonglong)]
            L.mmgap_server_poll.argtypes = [vp, ctypes.c_ulonglong, ctypes.POINTER(i),
                                            ctypes.POINTER(ctypes.c_double)]
            L.mmgap_server_stats.argtypes = [vp, ctypes.c_double, i, ctypes.POINTER(ServerStats)]
            L.mmgap_server_drain.argtypes = [vp]
            L.mmgap_server_stop.argtypes = [vp]
            for name in EXPORTS:
                if name not in ("mmgap_last_error",):
                    getattr(L, name).restype = i
            _lib = L
    return _lib


def _torch():
    import torch
    return torch


def _ptr(t):
    return None if t is None else ctypes.c_void_p(t.data_ptr())


def _stream(device) -> ctypes.c_void_p:
    torch = _torch()
    return ctypes.c_void_p(torch.cuda.current_stream(device).cuda_stream)


def qam_bits(qam: int) -> int:
    q = {4: 1, 16: 2, 64: 3}.get(int(qam))
    if q is None:
        raise ValueError(f"qam must be 4, 16 or 64 (got {qam})")
    return q


def linear_beta2(sweeps: int, beta0: float, beta1: float) -> np.ndarray:
    """Linear-in-beta anneal as the float32 table beta_t * log2(e) the library takes."""
    t = np.arange(sweeps, dtype=np.float64)
    b = np.full(sweeps, beta1) if sweeps == 1 else beta0 + (beta1 - beta0) * t / (sweeps - 1)
    return (b / math.log(2.0)).astype(np.float32)


def default_det_schedule(qam: int, n_rx: int, noise_var: float, sweeps: int) -> np.ndarray:
    """beta from 1/(4 c^2 n_rx) (cheapest uphill move accepted with e^-1) to
    1/sigma^2 (the posterior temperature of the Gaussian channel)."""
    c2 = 1.0 / (2.0 * (qam - 1) / 3.0)
    b0 = 1.0 / (4.0 * c2 * n_rx)
    b1 = max(1.0 / max(noise_var, 1e-6), b0)
    return linear_beta2(sweeps, b0, b1)


def default_vpp_schedule(qam: int, sweeps: int) -> np.ndarray:
    """beta from 0.1 to 4 in units of the perturbation step energy M c^2."""
    c2 = 1.0 / (2.0 * (qam - 1) / 3.0)
    step = qam * c2
    return linear_beta2(sweeps, 0.1 / step, 4.0 / step)


def _det_range(qam: int, n_rx: int, noise_var: float):
    c2 = 1.0 / (2.0 * (qam - 1) / 3.0)
    b0 = 1.0 / (4.0 * c2 * n_rx)
    return b0, max(1.0 / max(noise_var, 1e-6), b0)


def _vpp_range(qam: int):
    step = qam / (2.0 * (qam - 1) / 3.0)
    return 0.1 / step, 4.0 / step


TUNED_TABLE = os.path.join(_PKG, "tuned_schedules.json")
_tuned_cache = {}


def tuned_schedule(kind: int, n_rx: int, n_tx: int, qam: int, noise_var: float = 0.0,
                   table: str = TUNED_TABLE, any_formulation: bool = False) -> dict:
    """Schedule picked by the offline tuner (``python -m paper_2510_01579_amd.tune``)
    for a job: dict(chains, sweeps, init, beta2, stages, guesses, tuned,
    snr_bucket); stages >= 1 (detection only) selects moves around a guess with
    that many stages, 0 the binary encoding.  guesses is 0 for the binary
    encoding, GUESS_MMSE for moves around the MMSE guess (``detect_delta``),
    GUESS_SIC or GUESS_MMSE | GUESS_SIC (MMGaP-E) for ``detect_e``; batch jobs
    take stages and guesses (``det_job``).  The default is the tuner's choice by
    its cost model; any_formulation=True takes its choice by measured time per
    slot through the separate-launch entry points, where it timed candidates.

    Detection tables are bucketed by SNR = 10 log10(n_tx / noise_var) (per
    receive antenna, unit-energy symbols): the job takes the bucket of the
    smallest tuned SNR >= its own (the last bucket above the grid).  A class the
    table does not hold gets the reference schedule of its size (tuned=False).
    The temperature shape (r, m) ends the linear-in-beta anneal at m beta1 and
    starts it at r m beta1 (r = 0: at the default beta0)."""
    import json
    if table not in _tuned_cache:
        _tuned_cache[table] = {}
        if os.path.exists(table):
            with open(table) as fh:
                _tuned_cache[table] = json.load(fh).get("classes", {})
    name = f"{'det' if kind == KIND_DET else 'vpp'}-{n_rx}x{n_tx}-{int(qam)}"
    rec = _tuned_cache[table].get(name)
    bucket = None
    if rec is None:
        big = max(n_rx, n_tx) > 8
        sched = dict(chains=128 if big else 64, sweeps=400 if big else 200,
                     init=1 if (kind == KIND_DET and qam == 64) else 0, shape=[0.0, 1.0])
        tuned = False
    else:
        buckets = rec["buckets"]
        pick = buckets[-1]
        if kind == KIND_DET and buckets[0]["snr_db"] is not None:
            snr = 10.0 * math.log10(n_tx / max(float(noise_var), 1e-30))
            for b in buckets:                       # grid ascending
                if b["snr_db"] >= snr - 1e-3:
                    pick = b
                    break
        sched = dict(pick["tuned_any"] if any_formulation and "tuned_any" in pick
                     else pick["tuned"])
        bucket = pick["snr_db"]
        tuned = True
    b0, b1 = _det_range(qam, n_rx, noise_var) if kind == KIND_DET else _vpp_range(qam)
    r, m = sched.get("shape", [0.0, 1.0])
    end = m * b1
    start = b0 if r == 0.0 else max(b0, r * end)
    stages = int(sched.get("stages", 0))
    return dict(chains=int(sched["chains"]), sweeps=int(sched["sweeps"]),
                init=int(sched["init"]), beta2=linear_beta2(int(sched["sweeps"]),
                                                            min(start, end), end),
                stages=stages, guesses=int(sched.get("guesses", GUESS_MMSE if stages else 0)),
                tuned=tuned, snr_bucket=bucket)


class Context:
    """A library context bound to one HIP device (scratch, schedule ring, HBM budget)."""

    def __init__(self, device: int = 0, hbm_budget: int = 0):
        torch = _torch()
        if not torch.cuda.is_available():
            raise RuntimeError("no GPU visible: the MMGaP hot path runs only on a HIP device")
        self.device = int(device)
        self._h = ctypes.c_void_p()
        with torch.cuda.device(self.device):
            rc = lib().mmgap_create(ctypes.byref(self._h), self.device, int(hbm_budget))
        if rc != 0:
            raise MmgapError(rc, lib().mmgap_last_error(None).decode())

    def close(self):
        if self._h:
            lib().mmgap_destroy(self._h)
            self._h = ctypes.c_void_p()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def _check(self, rc: int):
        if rc != 0:
            raise MmgapError(rc, lib().mmgap_last_error(self._h).decode())

    def _dev(self):
        return _torch().device("cuda", self.device)

    def set_stage_launches(self, enable: bool = True):
        """MMGAP_OPT_STAGE_LAUNCHES: run detect_delta / detect_e as separate
        launches per stage (True) or in one launch where possible (False, the
        default); the outputs are identical."""
        self._check(lib().mmgap_set_option(self._h, OPT_STAGE_LAUNCHES, int(bool(enable))))

    def set_profiling(self, enable: bool = True):
        """(Re)start recording HIP events around the stages of every later call."""
        self._check(lib().mmgap_set_profiling(self._h, int(bool(enable))))

    def profile(self, max_calls: int = 256):
        """[(build_ms, anneal_ms, select_ms), ...] of the recorded calls, oldest first
        (waits for them)."""
        buf = (ctypes.c_float * (3 * max_calls))()
        rc = lib().mmgap_last_profile(self._h, buf, 3 * max_calls)
        if rc < 0:
            self._check(rc)
        return [tuple(float(v) for v in buf[i:i + 3]) for i in range(0, rc, 3)]

    # ------------------------------------------------------------------ helpers
    def _check_tensor(self, t, name, dtype, shape):
        torch = _torch()
        if t.device != self._dev():
            raise ValueError(f"{name} must be on {self._dev()} (got {t.device})")
        if t.dtype != dtype:
            raise ValueError(f"{name} must be {dtype} (got {t.dtype})")
        if tuple(t.shape) != tuple(shape):
            raise ValueError(f"{name} must have shape {tuple(shape)} (got {tuple(t.shape)})")
        if not t.is_contiguous():
            raise ValueError(f"{name} must be contiguous")
        return t

    @staticmethod
    def _schedule(chains, sweeps, beta2, seed, init, cim=None, inst_base=0):
        """A Schedule and the host objects it points to (keep them alive).  cim:
        None for Metropolis anneals, else a dict of CIM-CAC constants (missing
        keys from CIM_DEFAULTS; `sweeps` is then the number of Euler steps and
        beta2 may be None).  inst_base: Philox instance index of instance 0."""
        ib = int(inst_base)
        if not 0 <= ib <= 0xFFFFFFFF:
            raise ValueError("inst_base must fit in 32 bits")
        if cim is None:
            b = np.ascontiguousarray(np.asarray(beta2, dtype=np.float32).reshape(-1))
            if b.size != sweeps:
                raise ValueError(f"beta2 must have {sweeps} entries (got {b.size})")
            s = Schedule(int(chains), int(sweeps), b.ctypes.data_as(ctypes.POINTER(ctypes.c_float)),
                         int(seed) & 0xFFFFFFFFFFFFFFFF, int(init), DYN_METROPOLIS, None, ib)
            return s, b
        P = dict(CIM_DEFAULTS)
        unknown = set(cim) - set(P)
        if unknown:
            raise ValueError(f"unknown CIM constants {sorted(unknown)}")
        P.update(cim)
        c = CimParams(float(P["dt"]), int(P["f_mvm"]), float(P["p"]), float(P["a"]),
                      float(P["zeta"]), float(P["eps"]), float(P["amp0"]))
        s = Schedule(int(chains), int(sweeps), None, int(seed) & 0xFFFFFFFFFFFFFFFF, int(init),
                     DYN_CIM, ctypes.pointer(c), ib)
        return s, c

    def _problem(self, kind, H, y_or_u, qam, noise_var, tau):
        torch = _torch()
        if H.dim() != 3 or y_or_u.dim() != 3:
            raise ValueError("H must be [n_sc][n_rx][n_tx] and y/u [n_sc][n_sym][n_rx]")
        n_sc, n_rx, n_tx = H.shape
        n_sym = y_or_u.shape[1]
        self._check_tensor(H, "H", torch.complex64, (n_sc, n_rx, n_tx))
        self._check_tensor(y_or_u, "y_or_u", torch.complex64, (n_sc, n_sym, n_rx))
        qam_bits(qam)
        return Problem(kind, n_rx, n_tx, int(qam), n_sc, n_sym, float(noise_var), float(tau))

    # ------------------------------------------------------------------ entry points
    def build_ising(self, kind, H, y_or_u, qam, noise_var=0.0, tau=0.0, fallback=True,
                    dense=False, stream=None):
        """Couplings G [n_sc][K][K], fields f [n][K] (float32), fallback levels
        x_fb [n][K] (int8) and, if dense, J [n_sc][N][N], h [n][N], e_const [n]."""
        torch = _torch()
        p = self._problem(kind, H, y_or_u, qam, noise_var, tau)
        K = 2 * (p.n_tx if kind == KIND_DET else p.n_rx)
        q = qam_bits(qam) if kind == KIND_DET else 2
        N = K * q
        n = p.n_sc * p.n_sym
        dev = self._dev()
        out = dict(G=torch.empty((p.n_sc, K, K), dtype=torch.float32, device=dev),
                   f=torch.empty((n, K), dtype=torch.float32, device=dev))
        out["x_fb"] = torch.empty((n, K), dtype=torch.int8, device=dev) if fallback else None
        if dense:
            out["J"] = torch.empty((p.n_sc, N, N), dtype=torch.float32, device=dev)
            out["h"] = torch.empty((n, N), dtype=torch.float32, device=dev)
            out["e_const"] = torch.empty((n,), dtype=torch.float32, device=dev)
        st = stream if stream is not None else _stream(dev)
        self._check(lib().mmgap_build_ising(self._h, ctypes.byref(p), _ptr(H), _ptr(y_or_u),
                                            _ptr(out["G"]), _ptr(out["f"]), _ptr(out["x_fb"]),
                                            _ptr(out.get("J")), _ptr(out.get("h")),
                                            _ptr(out.get("e_const")), st))
        return out

    def solve(self, G, f, K, q, w, chains, sweeps, beta2, seed, x_fallback=None, inst_per_G=1,
              init=0, stream=None, cim=None, inst_base=0):
        """Best of `chains` anneals per instance.  Returns (spins int8 [n][K q],
        energy float32 [n], winning chain int32 [n])."""
        torch = _torch()
        n = f.shape[0]
        n_G = (n + inst_per_G - 1) // inst_per_G if n else 0
        self._check_tensor(f, "f", torch.float32, (n, K))
        self._check_tensor(G, "G", torch.float32, (n_G, K, K))
        if x_fallback is not None:
            self._check_tensor(x_fallback, "x_fallback", torch.int8, (n, K))
        wv = (ctypes.c_byte * len(w))(*[int(v) for v in w])
        if len(w) != q:
            raise ValueError("w must have q entries")
        dev = self._dev()
        spins = torch.empty((n, K * q), dtype=torch.int8, device=dev)
        E = torch.empty((n,), dtype=torch.float32, device=dev)
        win = torch.empty((n,), dtype=torch.int32, device=dev)
        s, keep = self._schedule(chains, sweeps, beta2, seed, init, cim, inst_base)
        st = stream if stream is not None else _stream(dev)
        self._check(lib().mmgap_solve(self._h, n, K, q, wv, _ptr(G), int(inst_per_G), _ptr(f),
                                      _ptr(x_fallback), ctypes.byref(s), _ptr(spins), _ptr(E),
                                      _ptr(win), st))
        del keep
        return spins, E, win

    def cim_chains(self, G, f, K, q, w, chains, steps, seed, cim=None, x_fallback=None,
                   inst_per_G=1, init=0, stream=None, inst_base=0):
        """Every CIM-CAC anneal's final state (mmgap_cim_chains).  Returns (spins
        int8 [n][chains][K q], energy float32 [n][chains], diverged uint8
        [n][chains])."""
        torch = _torch()
        n = f.shape[0]
        n_G = (n + inst_per_G - 1) // inst_per_G if n else 0
        self._check_tensor(f, "f", torch.float32, (n, K))
        self._check_tensor(G, "G", torch.float32, (n_G, K, K))
        if x_fallback is not None:
            self._check_tensor(x_fallback, "x_fallback", torch.int8, (n, K))
        if len(w) != q:
            raise ValueError("w must have q entries")
        wv = (ctypes.c_byte * len(w))(*[int(v) for v in w])
        dev = self._dev()
        spins = torch.empty((n, chains, K * q), dtype=torch.int8, device=dev)
        E = torch.empty((n, chains), dtype=torch.float32, device=dev)
        div = torch.empty((n, chains), dtype=torch.uint8, device=dev)
        s, keep = self._schedule(chains, steps, None, seed, init, {} if cim is None else cim,
                                 inst_base)
        st = stream if stream is not None else _stream(dev)
        self._check(lib().mmgap_cim_chains(self._h, n, K, q, wv, _ptr(G), int(inst_per_G), _ptr(f),
                                           _ptr(x_fallback), ctypes.byref(s), _ptr(spins), _ptr(E),
                                           _ptr(div), st))
        del keep
        return spins, E, div

    def detect(self, H, y, qam, noise_var, chains, sweeps, beta2, seed, init=0, metric=True,
               stream=None, cim=None, inst_base=0):
        """Uplink detection.  Returns (sym uint8 [n][n_tx], metric float32 [n] or None)."""
        torch = _torch()
        p = self._problem(KIND_DET, H, y, qam, noise_var, 0.0)
        n = p.n_sc * p.n_sym
        dev = self._dev()
        sym = torch.empty((n, p.n_tx), dtype=torch.uint8, device=dev)
        met = torch.empty((n,), dtype=torch.float32, device=dev) if metric else None
        s, keep = self._schedule(chains, sweeps, beta2, seed, init, cim, inst_base)
        st = stream if stream is not None else _stream(dev)
        self._check(lib().mmgap_detect(self._h, ctypes.byref(p), _ptr(H), _ptr(y),
                                       ctypes.byref(s), _ptr(sym), _ptr(met), st))
        del keep
        return sym, met

    def detect_noalloc(self, H, y, qam, noise_var, chains, sweeps, beta2, seed, init=0,
                       sym=None, metric=None, stream=None, cim=None, inst_base=0):
        """mmgap_detect_noalloc: detection whose scratch is the library's fixed
        per-device array (no device allocation inside the call).  `sym` (uint8
        [n][n_tx]) and `metric` (float32 [n]) may be given as preallocated
        outputs; otherwise they are allocated here, before the call.  Returns
        (sym, metric or None)."""
        torch = _torch()
        p = self._problem(KIND_DET, H, y, qam, noise_var, 0.0)
        n = p.n_sc * p.n_sym
        dev = self._dev()
        if sym is None:
            sym = torch.empty((n, p.n_tx), dtype=torch.uint8, device=dev)
        else:
            self._check_tensor(sym, "sym", torch.uint8, (n, p.n_tx))
        if metric is not None:
            self._check_tensor(metric, "metric", torch.float32, (n,))
        s, keep = self._schedule(chains, sweeps, beta2, seed, init, cim, inst_base)
        st = stream if stream is not None else _stream(dev)
        self._check(lib().mmgap_detect_noalloc(self._h, ctypes.byref(p), _ptr(H), _ptr(y),
                                               ctypes.byref(s), _ptr(sym), _ptr(metric), st))
        del keep
        return sym, metric

    def detect_delta(self, H, y, qam, noise_var, chains, sweeps, beta2, seed, stages=1,
                     guess=None, init=0, metric=True, stream=None, cim=None, inst_base=0):
        """Detection by moves around a guess (mmgap_detect_delta): `stages` anneals
        of the {-2, 0, 2}-move problem from the sliced MMSE estimate (or `guess`,
        int8 levels [n][2 n_tx]).  Returns (sym uint8 [n][n_tx], metric float32
        [n] or None)."""
        torch = _torch()
        p = self._problem(KIND_DET, H, y, qam, noise_var, 0.0)
        n = p.n_sc * p.n_sym
        if guess is not None:
            self._check_tensor(guess, "guess", torch.int8, (n, 2 * p.n_tx))
        dev = self._dev()
        sym = torch.empty((n, p.n_tx), dtype=torch.uint8, device=dev)
        met = torch.empty((n,), dtype=torch.float32, device=dev) if metric else None
        s, keep = self._schedule(chains, sweeps, beta2, seed, init, cim, inst_base)
        st = stream if stream is not None else _stream(dev)
        self._check(lib().mmgap_detect_delta(self._h, ctypes.byref(p), _ptr(H), _ptr(y),
                                             ctypes.byref(s), int(stages), _ptr(guess),
                                             _ptr(sym), _ptr(met), st))
        del keep
        return sym, met

    def detect_sic(self, H, y, qam, noise_var, metric=True, levels=False, order=False,
                   stream=None):
        """Ordered MMSE-SIC (mmgap_detect_sic).  Returns (sym uint8 [n][n_tx],
        metric float32 [n] or None, levels int8 [n][2 n_tx] or None, order int32
        [n_sc][n_tx] or None)."""
        torch = _torch()
        p = self._problem(KIND_DET, H, y, qam, noise_var, 0.0)
        n = p.n_sc * p.n_sym
        dev = self._dev()
        sym = torch.empty((n, p.n_tx), dtype=torch.uint8, device=dev)
        met = torch.empty((n,), dtype=torch.float32, device=dev) if metric else None
        lv = torch.empty((n, 2 * p.n_tx), dtype=torch.int8, device=dev) if levels else None
        od = torch.empty((p.n_sc, p.n_tx), dtype=torch.int32, device=dev) if order else None
        st = stream if stream is not None else _stream(dev)
        self._check(lib().mmgap_detect_sic(self._h, ctypes.byref(p), _ptr(H), _ptr(y), _ptr(sym),
                                           _ptr(met), _ptr(lv), _ptr(od), st))
        return sym, met, lv, od

    def detect_e(self, H, y, qam, noise_var, chains, sweeps, beta2, seed, stages=1, init=0,
                 metric=True, stream=None, cim=None, guesses=3, inst_base=0):
        """MMGaP-E (mmgap_detect_e): stages of moves from the MMSE and from the
        MMSE-SIC guess, the better answer (`guesses` selects one chain or both).
        Returns (sym uint8 [n][n_tx], metric float32 [n] or None, from_sic uint8
        [n])."""
        torch = _torch()
        p = self._problem(KIND_DET, H, y, qam, noise_var, 0.0)
        n = p.n_sc * p.n_sym
        dev = self._dev()
        sym = torch.empty((n, p.n_tx), dtype=torch.uint8, device=dev)
        met = torch.empty((n,), dtype=torch.float32, device=dev) if metric else None
        fs = torch.empty((n,), dtype=torch.uint8, device=dev)
        s, keep = self._schedule(chains, sweeps, beta2, seed, init, cim, inst_base)
        st = stream if stream is not None else _stream(dev)
        self._check(lib().mmgap_detect_e(self._h, ctypes.byref(p), _ptr(H), _ptr(y),
                                         ctypes.byref(s), int(stages), int(guesses), _ptr(sym),
                                         _ptr(met), _ptr(fs), st))
        del keep
        return sym, met, fs

    def vpp_precode(self, H, u, qam, chains, sweeps, beta2, seed, tau=0.0, want_x=True,
                    want_gamma=True, init=0, stream=None, cim=None, inst_base=0):
        """Downlink VPP.  Returns (v int8 [n][2 n_rx], x complex64 [n][n_tx] or None,
        gamma float32 [n] or None)."""
        torch = _torch()
        p = self._problem(KIND_VPP, H, u, qam, 0.0, tau)
        n = p.n_sc * p.n_sym
        dev = self._dev()
        v = torch.empty((n, 2 * p.n_rx), dtype=torch.int8, device=dev)
        x = torch.empty((n, p.n_tx), dtype=torch.complex64, device=dev) if want_x else None
        g = torch.empty((n,), dtype=torch.float32, device=dev) if want_gamma else None
        s, keep = self._schedule(chains, sweeps, beta2, seed, init, cim, inst_base)
        st = stream if stream is not None else _stream(dev)
        self._check(lib().mmgap_vpp_precode(self._h, ctypes.byref(p), _ptr(H), _ptr(u),
                                            ctypes.byref(s), _ptr(v), _ptr(x), _ptr(g), st))
        del keep
        return v, x, g

    # ------------------------------------------------------------------ batches
    def det_job(self, H, y, qam, noise_var, chains, sweeps, beta2, seed, init=0, metric=True,
                stages=0, inst_base=0, guesses=0, cim=None):
        """A detection job for ``plan_create`` with its output tensors allocated:
        outputs["sym"] uint8 [n][n_tx], outputs["metric"] float32 [n] or None.
        stages >= 1: detection by moves around the MMSE estimate (detect_delta),
        or with guesses (GUESS_MMSE, GUESS_SIC or both) as detect_e, and then
        outputs["from_sic"] uint8 [n].  cim: CIM-CAC constants (as for detect;
        `sweeps` Euler steps, beta2 None) for a CIM-CAC job."""
        torch = _torch()
        p = self._problem(KIND_DET, H, y, qam, noise_var, 0.0)
        n = p.n_sc * p.n_sym
        dev = self._dev()
        out = dict(sym=torch.empty((n, p.n_tx), dtype=torch.uint8, device=dev),
                   metric=torch.empty((n,), dtype=torch.float32, device=dev) if metric else None)
        if guesses:
            out["from_sic"] = torch.empty((n,), dtype=torch.uint8, device=dev)
        s, keep = self._schedule(chains, sweeps, beta2, seed, init, cim, inst_base)
        job = Job(p, s, _ptr(H).value, _ptr(y).value, _ptr(out["sym"]).value,
                  None if out["metric"] is None else _ptr(out["metric"]).value,
                  _ptr(out["from_sic"]).value if guesses else None, int(stages), int(guesses))
        return dict(job=job, keep=(H, y, keep), outputs=out)

    def vpp_job(self, H, u, qam, chains, sweeps, beta2, seed, tau=0.0, want_x=True,
                want_gamma=True, init=0, inst_base=0, cim=None):
        """A VPP job for ``plan_create``: outputs["v"] int8 [n][2 n_rx],
        outputs["x"] complex64 [n][n_tx] or None, outputs["gamma"] float32 [n] or None."""
        torch = _torch()
        p = self._problem(KIND_VPP, H, u, qam, 0.0, tau)
        n = p.n_sc * p.n_sym
        dev = self._dev()
        out = dict(v=torch.empty((n, 2 * p.n_rx), dtype=torch.int8, device=dev),
                   x=torch.empty((n, p.n_tx), dtype=torch.complex64, device=dev) if want_x else None,
                   gamma=torch.empty((n,), dtype=torch.float32, device=dev) if want_gamma else None)
        s, keep = self._schedule(chains, sweeps, beta2, seed, init, cim, inst_base)
        job = Job(p, s, _ptr(H).value, _ptr(u).value, _ptr(out["v"]).value,
                  None if out["x"] is None else _ptr(out["x"]).value,
                  None if out["gamma"] is None else _ptr(out["gamma"]).value)
        return dict(job=job, keep=(H, u, keep), outputs=out)

    def plan_create(self, jobs, graph=True, blocks=0, persistent=False):
        """A Plan running `jobs` (from det_job / vpp_job) in one batch launch
        (persistent: every Metropolis job through the persistent kernels)."""
        arr = (Job * max(len(jobs), 1))(*[j["job"] for j in jobs])
        h = ctypes.c_void_p()
        flags = (PLAN_GRAPH if graph else 0) | (PLAN_PERSISTENT if persistent else 0)
        self._check(lib().mmgap_plan_create(self._h, len(jobs), arr, flags, int(blocks),
                                            ctypes.byref(h)))
        return Plan(self, h, jobs)

    # ------------------------------------------------------------------ serving
    def server_start(self, max_inflight: int = 2, arena_bytes: int = 0, max_batch_jobs: int = 0):
        """Start the native serving loop (see mmgap_server_start)."""
        self._check(lib().mmgap_server_start(self._h, int(max_inflight), int(arena_bytes),
                                             int(max_batch_jobs)))
        self._server_jobs = {}

    def server_submit(self, job, stream=None) -> int:
        """Queue a job made by det_job / vpp_job; returns its id.  The job's
        tensors are kept alive until it is reported done."""
        st = stream if stream is not None else _stream(self._dev())
        jid = ctypes.c_ulonglong()
        self._check(lib().mmgap_server_submit(self._h, ctypes.byref(job["job"]), st,
                                              ctypes.byref(jid)))
        self.__dict__.setdefault("_server_jobs", {})[jid.value] = job
        return jid.value

    def server_poll(self, job_id: int):
        """(done, latency_us or None)."""
        done, lat = ctypes.c_int(), ctypes.c_double()
        rc = lib().mmgap_server_poll(self._h, int(job_id), ctypes.byref(done), ctypes.byref(lat))
        if done.value:
            self.__dict__.get("_server_jobs", {}).pop(int(job_id), None)
        self._check(rc)
        return bool(done.value), (lat.value if done.value else None)

    def server_stats(self, deadline_ms: float, reset: bool = False) -> dict:
        """Latency accounting of the completed jobs (mmgap_server_stats), in ms."""
        st = ServerStats()
        self._check(lib().mmgap_server_stats(self._h, float(deadline_ms) * 1e3,
                                             int(bool(reset)), ctypes.byref(st)))
        return {"completed": int(st.completed), "missed": int(st.missed),
                "p50_ms": st.p50_us / 1e3, "p99_ms": st.p99_us / 1e3, "max_ms": st.max_us / 1e3}

    def server_drain(self):
        self._check(lib().mmgap_server_drain(self._h))

    def server_stop(self):
        self._check(lib().mmgap_server_stop(self._h))
        self._server_jobs = {}


class Plan:
    """A batch of jobs compiled to one persistent launch (see mmgap_plan_create).
    Holds references to the jobs' tensors, which the launches read and write."""

    def __init__(self, ctx: Context, handle, jobs):
        self.ctx = ctx
        self._h = handle
        self.jobs = jobs

    def plan_launch(self, stream=None):
        st = stream if stream is not None else _stream(self.ctx._dev())
        self.ctx._check(lib().mmgap_plan_launch(self._h, st))

    launch = plan_launch

    def plan_info(self):
        """(work items, persistent workgroups)."""
        a, b = ctypes.c_int(), ctypes.c_int()
        self.ctx._check(lib().mmgap_plan_info(self._h, ctypes.byref(a), ctypes.byref(b)))
        return a.value, b.value

    info = plan_info

    def plan_destroy(self):
        if self._h:
            lib().mmgap_plan_destroy(self._h)
            self._h = ctypes.c_void_p()

    destroy = plan_destroy

    def __del__(self):
        try:
            self.plan_destroy()
        except Exception:
            pass


_default_ctx = {}


def context(device: int = 0) -> Context:
    """Process-wide default context of a device."""
    if device not in _default_ctx:
        _default_ctx[device] = Context(device)
    return _default_ctx[device]


def build_ising(*args, device: int = 0, **kw):
    return context(device).build_ising(*args, **kw)


def solve(*args, device: int = 0, **kw):
    return context(device).solve(*args, **kw)


def detect(*args, device: int = 0, **kw):
    return context(device).detect(*args, **kw)


def vpp_precode(*args, device: int = 0, **kw):
    return context(device).vpp_precode(*args, **kw)
