"""ctypes front end of the FP64 CPU oracle (``arna_oracle.c``).

TEST INFRASTRUCTURE ONLY.  The oracle is the plain reference that the GPU
path is checked against.  Only the test-suite, the smoke check and the
CPU-baseline leg of the benchmark may import it; the product package never
imports it and has no CPU fallback.

Float parameters are rounded through float32 before they reach the C code, so
that the oracle and the FP32 GPU path start from the same parameter values.
"""
from __future__ import annotations

import ctypes
import os
import subprocess
from dataclasses import dataclass, field

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "arna_oracle.c")
# ARNA_ORACLE_LIB names another build of the same source (the sanitizer test
# loads an ASan/UBSan build this way); it is used as it is, never rebuilt.
_LIB_OVERRIDE = os.environ.get("ARNA_ORACLE_LIB")
_LIB = os.path.join(_HERE, "liboracle.so")

MODE_RNA, MODE_ARNA = 0, 1
INIT_TRACKING, INIT_INFOSHARE = 0, 1
LIK_PATCH, LIK_POINT, LIK_POISSON = 0, 1, 2


def build(force: bool = True) -> str:
    """Compile the oracle with gcc (-O2, OpenMP over PEs)."""
    if force or not os.path.exists(_LIB):
        cmd = ["gcc", "-O2", "-fopenmp", "-std=gnu11", "-Wall", "-shared", "-fPIC",
               "-o", _LIB + ".tmp", _SRC, "-lm"]
        subprocess.run(cmd, check=True)
        os.replace(_LIB + ".tmp", _LIB)
    return _LIB


_lib = None


def lib():
    global _lib
    if _lib is None:
        if _LIB_OVERRIDE:
            _lib = ctypes.CDLL(_LIB_OVERRIDE)
            _declare(_lib)
            return _lib
        if not os.path.exists(_LIB) or os.path.getmtime(_LIB) < os.path.getmtime(_SRC):
            build()
        _lib = ctypes.CDLL(_LIB)
        _declare(_lib)
    return _lib


class _Config(ctypes.Structure):
    _fields_ = [
        ("n_filters", ctypes.c_uint32), ("n_pe", ctypes.c_uint32), ("n_per_pe", ctypes.c_uint32),
        ("width", ctypes.c_uint32), ("height", ctypes.c_uint32), ("patch", ctypes.c_uint32),
        ("mode", ctypes.c_int32), ("init_mode", ctypes.c_int32), ("lik_mode", ctypes.c_int32),
        ("fixed_ratio", ctypes.c_double), ("initial_ratio", ctypes.c_double),
        ("eff_cutoff", ctypes.c_double),
        ("psf_sigma", ctypes.c_double), ("background", ctypes.c_double),
        ("noise_sigma", ctypes.c_double), ("q", ctypes.c_double), ("sigma_I", ctypes.c_double),
        ("seed", ctypes.c_uint64), ("ring_groups", ctypes.c_uint32),
    ]


_TRACE_FIELDS = [
    # name, ctype, shape kind
    ("ring_pi", ctypes.c_uint32, "FM"), ("ring_pred", ctypes.c_uint32, "FM"),
    ("n_ex", ctypes.c_uint32, "F"), ("exch_off", ctypes.c_uint32, "FM"),
    ("src_map", ctypes.c_int64, "N"), ("lambda", ctypes.c_double, "N"),
    ("prop", ctypes.c_double, "5N"), ("ell", ctypes.c_double, "N"),
    ("Q", ctypes.c_uint32, "N"), ("T", ctypes.c_uint32, "FM"), ("V", ctypes.c_uint32, "FM"),
    ("anc", ctypes.c_uint32, "N"), ("state", ctypes.c_double, "5N"),
    ("L_pe", ctypes.c_double, "FM"), ("lstar", ctypes.c_double, "FM"),
    ("xhat_pe", ctypes.c_double, "FM5"), ("xhat", ctypes.c_double, "F5"),
    ("L_glob", ctypes.c_double, "F"), ("P", ctypes.c_uint32, "FM"),
    ("pe_eff", ctypes.c_double, "F"), ("log_z", ctypes.c_double, "F"),
    ("n_ex_next", ctypes.c_uint32, "F"), ("lineage", ctypes.c_int32, "N"),
    ("amb", ctypes.c_uint32, "N"), ("ell_alt", ctypes.c_double, "N3"),
]


class _Trace(ctypes.Structure):
    _fields_ = [(name, ctypes.POINTER(ct)) for name, ct, _ in _TRACE_FIELDS]


def _declare(L):
    u32, u64, i32 = ctypes.c_uint32, ctypes.c_uint64, ctypes.c_int
    P32 = ctypes.POINTER(ctypes.c_uint32)
    L.orc_philox.argtypes = [P32, P32, P32]
    L.orc_ring.argtypes = [u64, u32, u32, u32, i32, P32, P32, P32]
    L.orc_ring_groups.argtypes = [u64, u32, u32, u32, u32, P32, P32, P32]
    L.orc_fixed_nex.argtypes = [ctypes.c_double, u32]
    L.orc_fixed_nex.restype = u32
    L.orc_nex.argtypes = [P32, u32, u32, i32, ctypes.c_double, ctypes.c_double,
                          ctypes.c_double, i32]
    L.orc_nex.restype = u32
    L.orc_exchange_offset.argtypes = [u64, u32, u32, u32, u32]
    L.orc_exchange_offset.restype = u32
    L.orc_selected_slot.argtypes = [u32, u32, u32, u32]
    L.orc_selected_slot.restype = u32
    L.orc_resample_offset.argtypes = [u64, u32, u32, u32, u32]
    L.orc_resample_offset.restype = u32
    L.orc_resample.argtypes = [P32, u32, u32, P32]
    L.orc_resample.restype = i32
    L.orc_qmax.argtypes = [u32]
    L.orc_qmax.restype = u32
    L.orc_create.argtypes = [ctypes.POINTER(_Config), ctypes.POINTER(ctypes.c_double)]
    L.orc_create.restype = ctypes.c_void_p
    L.orc_destroy.argtypes = [ctypes.c_void_p]
    L.orc_set_state.argtypes = [ctypes.c_void_p, ctypes.POINTER(ctypes.c_double),
                                ctypes.POINTER(ctypes.c_double), u32]
    L.orc_get_state.argtypes = [ctypes.c_void_p, ctypes.POINTER(ctypes.c_double),
                                ctypes.POINTER(ctypes.c_double), P32]
    L.orc_set_lineage.argtypes = [ctypes.c_void_p, ctypes.POINTER(ctypes.c_int32)]
    L.orc_step.argtypes = [ctypes.c_void_p, ctypes.POINTER(ctypes.c_float),
                           ctypes.POINTER(_Trace)]
    L.orc_step.restype = i32
    L.orc_num_threads.restype = i32
    L.orc_set_num_threads.restype = None
    L.orc_set_num_threads.argtypes = [i32]
    PD = ctypes.POINTER(ctypes.c_double)
    L.orc_normals.argtypes = [u64, u32, u32, u32, PD]
    L.orc_propagate.argtypes = [PD, PD, ctypes.c_double, ctypes.c_double, PD]
    L.orc_loglik.argtypes = [ctypes.POINTER(_Config), ctypes.POINTER(ctypes.c_float), u32, PD]
    L.orc_loglik.restype = ctypes.c_double
    PI32 = ctypes.POINTER(ctypes.c_int32)
    PF = ctypes.POINTER(ctypes.c_float)
    L.orc_grad.argtypes = [ctypes.POINTER(_Config), PD, PF, u32, PD, PD, P32, P32, PI32]
    L.orc_grad.restype = i32
    L.orc_replay.argtypes = [ctypes.POINTER(_Config), PD, ctypes.c_double, PF, u32, P32, P32,
                             PI32, PD]
    L.orc_replay.restype = i32
    L.orc_set_ambiguity.argtypes = [ctypes.c_void_p, ctypes.c_double, ctypes.c_double]
    L.orc_pe_update.argtypes = [ctypes.POINTER(_Config), u32, u32, u32, u32, PD, PD, PD, PD, PD,
                                PD, P32, P32, P32, P32]
    L.orc_pe_update.restype = i32
    L.orc_master.argtypes = [ctypes.POINTER(_Config), PD, PD, PD, PD, P32, PD, PD, P32]


def _p(a, ct):
    return a.ctypes.data_as(ctypes.POINTER(ct))


def _f32(x) -> float:
    return float(np.float32(x))


# ------------------------------------------------------------------ primitives
def philox(ctr, key) -> np.ndarray:
    c = np.asarray(ctr, dtype=np.uint32).copy()
    k = np.asarray(key, dtype=np.uint32).copy()
    o = np.zeros(4, dtype=np.uint32)
    lib().orc_philox(_p(c, ctypes.c_uint32), _p(k, ctypes.c_uint32), _p(o, ctypes.c_uint32))
    return o


def ring(seed: int, f: int, k: int, M: int, mode: int = MODE_ARNA):
    pi = np.zeros(M, np.uint32)
    pred = np.zeros(M, np.uint32)
    succ = np.zeros(M, np.uint32)
    lib().orc_ring(seed, f, k, M, mode, _p(pi, ctypes.c_uint32), _p(pred, ctypes.c_uint32),
                   _p(succ, ctypes.c_uint32))
    return pi, pred, succ


def ring_groups(seed: int, f: int, k: int, M: int, G: int):
    """Hardware-aware ring: PE m of filter f in group (f M + m) mod G."""
    pi = np.zeros(M, np.uint32)
    pred = np.zeros(M, np.uint32)
    succ = np.zeros(M, np.uint32)
    lib().orc_ring_groups(seed, f, k, M, G, _p(pi, ctypes.c_uint32), _p(pred, ctypes.c_uint32),
                          _p(succ, ctypes.c_uint32))
    return pi, pred, succ


def fixed_nex(ratio: float, n_p: int) -> int:
    return int(lib().orc_fixed_nex(_f32(ratio), n_p))


def nex(P, n_p: int, mode: int = MODE_ARNA, fixed_ratio: float = 0.1,
        initial_ratio: float = 0.1, cutoff: float = 0.99, first: bool = False) -> int:
    P = np.ascontiguousarray(P, dtype=np.uint32)
    return int(lib().orc_nex(_p(P, ctypes.c_uint32), len(P), n_p, mode, _f32(fixed_ratio),
                             _f32(initial_ratio), _f32(cutoff), int(first)))


def exchange_offset(seed: int, f: int, k: int, m: int, n_p: int) -> int:
    return int(lib().orc_exchange_offset(seed, f, k, m, n_p))


def selected_slot(t: int, c: int, n_p: int, n_ex: int) -> int:
    return int(lib().orc_selected_slot(t, c, n_p, n_ex))


def resample_offset(seed: int, f: int, k: int, m: int, T: int) -> int:
    return int(lib().orc_resample_offset(seed, f, k, m, T))


def qmax(n_p: int) -> int:
    return int(lib().orc_qmax(n_p))


def resample(Q, V: int) -> np.ndarray:
    Q = np.ascontiguousarray(Q, dtype=np.uint32)
    anc = np.zeros(len(Q), np.uint32)
    rc = lib().orc_resample(_p(Q, ctypes.c_uint32), len(Q), V, _p(anc, ctypes.c_uint32))
    if rc != 0:
        raise ValueError("orc_resample: total weight is zero or V >= T")
    return anc


def normals(seed: int, f: int, k: int, j: int) -> np.ndarray:
    """The five standard normals of slot j (index within the filter) at step k."""
    e = np.zeros(5)
    lib().orc_normals(seed, f, k, j, _p(e, ctypes.c_double))
    return e


def propagate(state5, eps5, q: float, sigma_I: float) -> np.ndarray:
    a = np.ascontiguousarray(state5, dtype=np.float64)
    e = np.ascontiguousarray(eps5, dtype=np.float64)
    o = np.zeros(5)
    lib().orc_propagate(_p(a, ctypes.c_double), _p(e, ctypes.c_double), q, sigma_I,
                        _p(o, ctypes.c_double))
    return o


def loglik(cfg, frame, f: int, state5) -> float:
    if isinstance(cfg, dict):
        cfg = OracleConfig.from_dict(cfg)
    c = cfg.to_c()
    fr = np.ascontiguousarray(frame, dtype=np.float32)
    st = np.ascontiguousarray(state5, dtype=np.float64)
    return float(lib().orc_loglik(ctypes.byref(c), _p(fr, ctypes.c_float), f,
                                  _p(st, ctypes.c_double)))


def num_threads() -> int:
    return int(lib().orc_num_threads())


def set_num_threads(n: int) -> None:
    """OpenMP threads of later oracle calls."""
    lib().orc_set_num_threads(int(n))


# ------------------------------------------------------------------ filter
@dataclass
class OracleConfig:
    n_filters: int = 1
    n_pe: int = 4
    n_per_pe: int = 256
    width: int = 128
    height: int = 128
    patch: int = 9
    mode: int = MODE_RNA
    init_mode: int = INIT_TRACKING
    lik_mode: int = LIK_PATCH
    fixed_ratio: float = 0.1
    initial_ratio: float = 0.1
    eff_cutoff: float = 0.99
    psf_sigma: float = 1.5
    background: float = 5.0
    noise_sigma: float = 2.0
    q: float = 0.5
    sigma_I: float = 0.5
    seed: int = 1
    ring_groups: int = 0
    extra: dict = field(default_factory=dict)

    @classmethod
    def from_dict(cls, d: dict) -> "OracleConfig":
        names = {f for f in cls.__dataclass_fields__ if f != "extra"}
        return cls(**{k: v for k, v in d.items() if k in names})

    def to_c(self, psf_sigma: float | None = None, q: float | None = None) -> _Config:
        """psf_sigma / q, when given, are passed unrounded (finite differences)."""
        return _Config(self.n_filters, self.n_pe, self.n_per_pe, self.width, self.height,
                       self.patch, self.mode, self.init_mode, self.lik_mode,
                       _f32(self.fixed_ratio), _f32(self.initial_ratio), _f32(self.eff_cutoff),
                       _f32(self.psf_sigma) if psf_sigma is None else float(psf_sigma),
                       _f32(self.background), _f32(self.noise_sigma),
                       _f32(self.q) if q is None else float(q), _f32(self.sigma_I), self.seed,
                       self.ring_groups)

    @property
    def N(self) -> int:
        return self.n_filters * self.n_pe * self.n_per_pe


class Oracle:
    """M PEs x N_p particles per filter, F filters, all in FP64 on the CPU."""

    def __init__(self, cfg, truth):
        if isinstance(cfg, dict):
            cfg = OracleConfig.from_dict(cfg)
        self.cfg = cfg
        self._c = cfg.to_c()
        t = np.ascontiguousarray(np.asarray(truth, dtype=np.float32).astype(np.float64)
                                 .reshape(cfg.n_filters, 5))
        self._h = lib().orc_create(ctypes.byref(self._c), _p(t, ctypes.c_double))
        if not self._h:
            raise ValueError("orc_create rejected the configuration")

    def __del__(self):
        h = getattr(self, "_h", None)
        if h:
            lib().orc_destroy(h)
            self._h = None

    def set_state(self, state, L=None, k: int = 0):
        N = self.cfg.N
        s = np.ascontiguousarray(np.asarray(state, dtype=np.float64).reshape(5, N))
        Lp = None
        if L is not None:
            Larr = np.ascontiguousarray(np.asarray(L, dtype=np.float64).reshape(-1))
            Lp = _p(Larr, ctypes.c_double)
        lib().orc_set_state(self._h, _p(s, ctypes.c_double), Lp, k)

    def set_ambiguity(self, eps_rel: float, eps_abs: float):
        """From the next step on, trace which patch centres a coordinate error
        of eps_rel * max(|x|, 1) + eps_abs could move (``amb``) and the
        likelihoods at the other centres (``ell_alt``); 0, 0 turns it off."""
        lib().orc_set_ambiguity(self._h, float(eps_rel), float(eps_abs))

    def set_lineage(self, tag):
        t = np.ascontiguousarray(np.asarray(tag, dtype=np.int32).reshape(-1))
        lib().orc_set_lineage(self._h, _p(t, ctypes.c_int32))

    def get_state(self):
        N = self.cfg.N
        s = np.zeros((5, N), np.float64)
        L = np.zeros(self.cfg.n_filters * self.cfg.n_pe, np.float64)
        k = np.zeros(1, np.uint32)
        lib().orc_get_state(self._h, _p(s, ctypes.c_double), _p(L, ctypes.c_double),
                            _p(k, ctypes.c_uint32))
        return s, L.reshape(self.cfg.n_filters, self.cfg.n_pe), int(k[0])

    def step(self, frame, trace=True, want=None):
        """Run one iteration on ``frame`` ([H][W] patch mode, [F][2] point mode).

        Returns a dict of trace arrays (all of them, or the names in ``want``)."""
        c = self.cfg
        F, M, N = c.n_filters, c.n_pe, c.N
        fr = np.ascontiguousarray(np.asarray(frame, dtype=np.float32))
        shapes = {"F": (F,), "FM": (F, M), "N": (N,), "5N": (5, N), "FM5": (F, M, 5),
                  "F5": (F, 5), "N3": (N, 3)}
        dt = {ctypes.c_uint32: np.uint32, ctypes.c_int64: np.int64, ctypes.c_double: np.float64,
              ctypes.c_int32: np.int32}
        tr = _Trace()
        out = {}
        if trace:
            for name, ct, kind in _TRACE_FIELDS:
                if want is not None and name not in want:
                    continue
                a = np.zeros(shapes[kind], dt[ct])
                out[name] = a
                setattr(tr, name, _p(a, ct))
        rc = lib().orc_step(self._h, _p(fr, ctypes.c_float), ctypes.byref(tr) if trace else None)
        out["status"] = int(rc)
        return out


def pe_update(cfg, f: int, k: int, m: int, lam, ell, prop) -> dict:
    """Steps 6-7 of one PE from its carried log-weights, log-likelihoods and
    propagated particles ([5][n_p]), exactly as ``Oracle.step`` runs them."""
    if isinstance(cfg, dict):
        cfg = OracleConfig.from_dict(cfg)
    c = cfg.to_c()
    lam = np.ascontiguousarray(lam, dtype=np.float64)
    ell = np.ascontiguousarray(ell, dtype=np.float64)
    prop = np.ascontiguousarray(prop, dtype=np.float64)
    n_p = len(lam)
    xm = np.zeros(5)
    L = np.zeros(1)
    lstar = np.zeros(1)
    Q = np.zeros(n_p, np.uint32)
    T = np.zeros(1, np.uint32)
    V = np.zeros(1, np.uint32)
    anc = np.zeros(n_p, np.uint32)
    PD = ctypes.c_double
    st = lib().orc_pe_update(ctypes.byref(c), f, k, m, n_p, _p(lam, PD), _p(ell, PD),
                             _p(prop, PD), _p(xm, PD), _p(L, PD), _p(lstar, PD),
                             _p(Q, ctypes.c_uint32), _p(T, ctypes.c_uint32),
                             _p(V, ctypes.c_uint32), _p(anc, ctypes.c_uint32))
    return {"xhat_pe": xm, "L_pe": float(L[0]), "lstar": float(lstar[0]), "Q": Q,
            "T": int(T[0]), "V": int(V[0]), "anc": anc, "status": int(st)}


def master(cfg, L_pe, xhat_pe) -> dict:
    """Steps 9-10 of one filter from its PE log masses [M] and estimates [M][5]."""
    if isinstance(cfg, dict):
        cfg = OracleConfig.from_dict(cfg)
    c = cfg.to_c()
    M = cfg.n_pe
    L = np.ascontiguousarray(L_pe, dtype=np.float64)
    xm = np.ascontiguousarray(xhat_pe, dtype=np.float64)
    Lg = np.zeros(1)
    xh = np.zeros(5)
    P = np.zeros(M, np.uint32)
    eff = np.zeros(1)
    lz = np.zeros(1)
    nx = np.zeros(1, np.uint32)
    PD = ctypes.c_double
    lib().orc_master(ctypes.byref(c), _p(L, PD), _p(xm, PD), _p(Lg, PD), _p(xh, PD),
                     _p(P, ctypes.c_uint32), _p(eff, PD), _p(lz, PD), _p(nx, ctypes.c_uint32))
    return {"L_glob": float(Lg[0]), "xhat": xh, "P": P, "pe_eff": float(eff[0]),
            "log_z": float(lz[0]), "n_ex_next": int(nx[0])}


# ------------------------------------------------------------------ gradient
@dataclass
class Tape:
    """Discrete choices of a run: N_ex [K][F], ancestors [K][N], patch
    centres [K][N][2] (INT32_MIN where a patch misses the image)."""
    n_ex: np.ndarray
    anc: np.ndarray
    centre: np.ndarray


def _frames_k(frames) -> tuple:
    fr = np.ascontiguousarray(frames, dtype=np.float32)
    return fr, fr.shape[0]


def grad(cfg, truth, frames):
    """Run K = len(frames) iterations from the start; return J [F] (the
    estimate of log p(z_1..z_K) per filter), dJ/dtheta [F][3] with
    theta = (psf_sigma, I0, q) and the discrete choices held fixed, and the
    tape of those choices."""
    if isinstance(cfg, dict):
        cfg = OracleConfig.from_dict(cfg)
    c = cfg.to_c()
    fr, K = _frames_k(frames)
    t = np.ascontiguousarray(truth, dtype=np.float64)
    F, N = cfg.n_filters, cfg.N
    J = np.zeros(F)
    dJ = np.zeros((F, 3))
    tape = Tape(np.zeros((K, F), np.uint32), np.zeros((K, N), np.uint32),
                np.zeros((K, N, 2), np.int32))
    rc = lib().orc_grad(ctypes.byref(c), _p(t, ctypes.c_double), _p(fr, ctypes.c_float), K,
                        _p(J, ctypes.c_double), _p(dJ, ctypes.c_double),
                        _p(tape.n_ex, ctypes.c_uint32), _p(tape.anc, ctypes.c_uint32),
                        _p(tape.centre, ctypes.c_int32))
    if rc != 0:
        raise RuntimeError(f"orc_grad failed ({rc})")
    return J, dJ, tape


def replay(cfg, truth, frames, tape: Tape, psf_sigma=None, q=None, dI0: float = 0.0):
    """J [F] with the choices of `tape`; psf_sigma and q unrounded when given,
    every starting intensity shifted by dI0."""
    if isinstance(cfg, dict):
        cfg = OracleConfig.from_dict(cfg)
    c = cfg.to_c(psf_sigma=psf_sigma, q=q)
    fr, K = _frames_k(frames)
    t = np.ascontiguousarray(truth, dtype=np.float64)
    J = np.zeros(cfg.n_filters)
    rc = lib().orc_replay(ctypes.byref(c), _p(t, ctypes.c_double), float(dI0),
                          _p(fr, ctypes.c_float), K, _p(tape.n_ex, ctypes.c_uint32),
                          _p(tape.anc, ctypes.c_uint32), _p(tape.centre, ctypes.c_int32),
                          _p(J, ctypes.c_double))
    if rc != 0:
        raise RuntimeError(f"orc_replay failed ({rc})")
    return J
