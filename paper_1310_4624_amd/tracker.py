"""Python face of the C interface: a Tracker object over pf_ctx and the
device integer stages as functions.  PyTorch supplies device memory (tensor
data pointers) and the stream; all filter work runs in libarna.so."""
from __future__ import annotations

import ctypes

import numpy as np

from . import _native as nat

CONFIG_KEYS = ("n_filters", "n_pe", "n_per_pe", "width", "height", "patch", "mode",
               "init_mode", "lik_mode", "fixed_ratio", "initial_ratio", "eff_cutoff",
               "psf_sigma", "background", "noise_sigma", "q", "sigma_I", "seed", "ring_groups",
               "block_size", "launch", "pes_per_wg")

DEFAULTS = dict(n_filters=1, n_pe=4, n_per_pe=256, width=128, height=128, patch=9,
                mode=nat.PF_MODE_RNA, init_mode=nat.PF_INIT_TRACKING, lik_mode=nat.PF_LIK_PATCH,
                fixed_ratio=0.1, initial_ratio=0.1, eff_cutoff=0.99, psf_sigma=1.5,
                background=5.0, noise_sigma=2.0, q=0.5, sigma_I=0.5, seed=1, ring_groups=0,
                block_size=0, launch=nat.PF_LAUNCH_AUTO, pes_per_wg=0)


TRAJ_RECORD_BYTES = ctypes.sizeof(nat.pf_master_t)


def trajectory(buf, n_steps: int, n_filters: int) -> dict:
    """Decode the master steps pf_run_traj wrote ([n_steps][F] pf_master_t,
    a CUDA uint8 tensor or host bytes) into arrays indexed [step][filter]."""
    raw = buf[:n_steps * n_filters * TRAJ_RECORD_BYTES]
    raw = raw.cpu().numpy() if hasattr(raw, "cpu") else np.asarray(raw, np.uint8)
    dt = np.dtype([("xhat", "<f8", 5), ("log_mass_glob", "<f8"), ("pe_eff", "<f8"),
                   ("log_z_inc", "<f8"), ("n_ex", "<u4"), ("n_ex_next", "<u4"),
                   ("step", "<u8")])
    assert dt.itemsize == TRAJ_RECORD_BYTES
    rec = np.frombuffer(raw.tobytes(), dtype=dt).reshape(n_steps, n_filters)
    return {k: rec[k].copy() for k in dt.names}


def _ptr(a: np.ndarray):
    return ctypes.c_void_p(a.ctypes.data)


def make_config(cfg: dict, stream=None, debug: int = 0) -> nat.pf_config:
    d = dict(DEFAULTS)
    d.update({k: v for k, v in cfg.items() if k in CONFIG_KEYS})
    c = nat.pf_config()
    c.struct_size = ctypes.sizeof(nat.pf_config)
    for k in CONFIG_KEYS:
        setattr(c, k, d[k])
    c.debug = debug
    c.stream = stream
    return c


def _torch_stream():
    import torch
    return ctypes.c_void_p(torch.cuda.current_stream().cuda_stream)


def _dev_ptr(t, what: str):
    import torch
    if not isinstance(t, torch.Tensor) or not t.is_cuda:
        raise TypeError(f"{what} must be a CUDA (HIP) tensor")
    if t.dtype != torch.float32 or not t.is_contiguous():
        raise TypeError(f"{what} must be contiguous float32")
    return ctypes.c_void_p(t.data_ptr())


class Tracker:
    """F independent filters, each of M PEs x N_p particles, on one GPU."""

    def __init__(self, cfg: dict, truth, debug: int = 0, stream=None):
        d = dict(DEFAULTS)
        d.update(cfg)
        self.cfg = d
        self.F, self.M, self.np_ = d["n_filters"], d["n_pe"], d["n_per_pe"]
        self.N = self.F * self.M * self.np_
        self._stream = stream if stream is not None else _torch_stream()
        self._c = make_config(d, stream=self._stream, debug=debug)
        t = np.ascontiguousarray(np.asarray(truth, dtype=np.float32).reshape(self.F, 5))
        h = ctypes.c_void_p()
        rc = nat.lib().pf_init(ctypes.byref(self._c),
                               t.ctypes.data_as(ctypes.POINTER(ctypes.c_float)), ctypes.byref(h))
        nat.check(rc, "pf_init")
        self._h = h

    def frame_numel(self) -> int:
        """Floats one frame must hold: [H][W] (patch) or [F][2] (point)."""
        if self.cfg["lik_mode"] == nat.PF_LIK_POINT:
            return 2 * self.F
        return self.cfg["width"] * self.cfg["height"]

    # ------------------------------------------------------------ the path
    def step(self, frame) -> None:
        if frame.numel() != self.frame_numel():
            raise ValueError(f"frame has {frame.numel()} values, expected {self.frame_numel()}")
        nat.check(nat.lib().pf_step(self._h, _dev_ptr(frame, "frame")), "pf_step")

    def run(self, frames, n_steps: int | None = None) -> None:
        """Consecutive iterations over frames[0], frames[1], ... (first axis)."""
        n = frames.shape[0] if n_steps is None else n_steps
        if n > frames.shape[0]:
            raise ValueError("more steps than frames")
        stride = int(np.prod(frames.shape[1:]))
        if stride != self.frame_numel():
            raise ValueError(f"frames hold {stride} values each, expected {self.frame_numel()}")
        nat.check(nat.lib().pf_run(self._h, _dev_ptr(frames, "frames"), n, stride), "pf_run")

    def run_traj(self, frames, traj, n_steps: int | None = None) -> None:
        """Like run(); the master step of every iteration (Alg. 3 steps 9-10)
        goes to ``traj``, a CUDA uint8 tensor of at least n_steps * F *
        TRAJ_RECORD_BYTES bytes, without a host synchronization (read it back
        with ``trajectory``)."""
        import torch
        n = frames.shape[0] if n_steps is None else n_steps
        if n > frames.shape[0]:
            raise ValueError("more steps than frames")
        stride = int(np.prod(frames.shape[1:]))
        if stride != self.frame_numel():
            raise ValueError(f"frames hold {stride} values each, expected {self.frame_numel()}")
        need = n * self.F * TRAJ_RECORD_BYTES
        if (not isinstance(traj, torch.Tensor) or not traj.is_cuda or traj.dtype != torch.uint8
                or not traj.is_contiguous() or traj.numel() < need):
            raise TypeError(f"traj must be a contiguous CUDA uint8 tensor of >= {need} bytes")
        nat.check(nat.lib().pf_run_traj(self._h, _dev_ptr(frames, "frames"), n, stride,
                                        ctypes.c_void_p(traj.data_ptr())), "pf_run_traj")

    def run_timed(self, frames, n_steps: int | None = None) -> np.ndarray:
        """Like run(); returns each iteration's duration in ms (HIP events on
        the context's stream, recorded by the library around its launches)."""
        n = frames.shape[0] if n_steps is None else n_steps
        if n > frames.shape[0]:
            raise ValueError("more steps than frames")
        stride = int(np.prod(frames.shape[1:]))
        if stride != self.frame_numel():
            raise ValueError(f"frames hold {stride} values each, expected {self.frame_numel()}")
        out = np.zeros(n, np.float32)
        nat.check(nat.lib().pf_run_timed(self._h, _dev_ptr(frames, "frames"), n, stride,
                                         out.ctypes.data_as(ctypes.POINTER(ctypes.c_float))),
                  "pf_run_timed")
        return out

    def multi_iteration(self) -> bool:
        """Whether run() may use multi-iteration launches (pf_run_info)."""
        v = ctypes.c_uint32()
        nat.check(nat.lib().pf_run_info(self._h, ctypes.byref(v)), "pf_run_info")
        return bool(v.value)

    def exchange(self, src_map=None) -> None:
        p = None
        if src_map is not None:
            import torch
            if src_map.dtype != torch.int64 or not src_map.is_cuda or src_map.numel() < self.N:
                raise TypeError("src_map must be a CUDA int64 tensor with N elements")
            p = ctypes.c_void_p(src_map.data_ptr())
        nat.check(nat.lib().pf_exchange(self._h, p), "pf_exchange")

    def grad_begin(self, max_steps: int) -> None:
        """Record the next max_steps iterations for grad_end."""
        nat.check(nat.lib().pf_grad_begin(self._h, int(max_steps)), "pf_grad_begin")

    def grad_end(self, frames) -> dict:
        """Reverse sweep over the recorded iterations (frames: the same frames,
        first axis = iteration).  Returns J [F] (estimate of the log marginal
        likelihood of the recorded frames) and grad [F][3], the derivatives
        of J in (psf_sigma, I0, q) with the discrete choices held fixed."""
        F = self.F
        out = np.zeros((F, 4))
        ptr = out.ctypes.data_as(ctypes.POINTER(ctypes.c_double))
        if frames is None or frames.shape[0] == 0:
            nat.check(nat.lib().pf_grad_end(self._h, None, 0, ptr), "pf_grad_end")
        else:
            stride = int(np.prod(frames.shape[1:]))
            if stride != self.frame_numel():
                raise ValueError(f"frames hold {stride} values each, expected {self.frame_numel()}")
            nat.check(nat.lib().pf_grad_end(self._h, _dev_ptr(frames, "frames"), stride, ptr),
                      "pf_grad_end")
        return dict(J=out[:, 0].copy(), grad=out[:, 1:].copy())

    def grad_value(self) -> np.ndarray:
        """While recording: J [F] over the iterations recorded so far."""
        out = np.zeros(self.F)
        nat.check(nat.lib().pf_grad_value(self._h, out.ctypes.data_as(
            ctypes.POINTER(ctypes.c_double))), "pf_grad_value")
        return out

    def estimate(self, raise_numeric: bool = True) -> dict:
        F, M = self.F, self.M
        out = dict(x_global=np.zeros((F, 5)), x_pe=np.zeros((F, M, 5)),
                   log_mass_pe=np.zeros((F, M)), log_mass_glob=np.zeros(F), pe_eff=np.zeros(F),
                   n_ex=np.zeros(F, np.uint32), n_ex_next=np.zeros(F, np.uint32),
                   log_z_inc=np.zeros(F))
        e = nat.pf_estimate_t()
        for k, a in out.items():
            ct = ctypes.c_uint32 if a.dtype == np.uint32 else ctypes.c_double
            setattr(e, k, a.ctypes.data_as(ctypes.POINTER(ct)))
        rc = nat.lib().pf_estimate(self._h, ctypes.byref(e))
        out["step"] = int(e.step)
        out["status"] = rc
        if rc != nat.PF_OK and (rc != nat.PF_ENUMERIC or raise_numeric):
            nat.check(rc, "pf_estimate")
        return out

    # ------------------------------------------------------------ debug
    def debug_get(self, which: str) -> np.ndarray:
        code = nat.DBG[which]
        n = nat.lib().pf_debug_size(self._h, code)
        if n == 0:
            raise nat.PFError(nat.PF_ESTATE, f"debug buffer {which} not kept (debug flags)")
        F, M, N = self.F, self.M, self.N
        shapes = dict(state=((5, N), np.float32), logmass=((F, M), np.float64),
                      ring=((F, M), np.uint32), nex=((F,), np.uint32), src=((N,), np.int64),
                      prop=((5, N), np.float32), ell=((N,), np.float32), q=((N,), np.uint32),
                      ancestors=((N,), np.uint32), v=((F, M), np.uint32),
                      lam=((N,), np.float32), lineage=((N,), np.int32))
        if which == "pe_records":
            a = (nat.pf_pe_record * (F * M))()
            nat.check(nat.lib().pf_debug_get(self._h, code, ctypes.cast(a, ctypes.c_void_p), n),
                      "pf_debug_get")
            return np.array([(r.log_mass, *r.xhat, r.lstar, r.total_q) for r in a]).reshape(F, M, 8)
        shape, dt = shapes[which]
        a = np.zeros(shape, dt)
        assert a.nbytes == n, (which, a.nbytes, n)
        nat.check(nat.lib().pf_debug_get(self._h, code, _ptr(a), n), "pf_debug_get")
        return a

    def set_state(self, state, log_mass=None, step: int = 0) -> None:
        s = np.ascontiguousarray(np.asarray(state, dtype=np.float32).reshape(5, self.N))
        L = None
        if log_mass is not None:
            L = np.ascontiguousarray(np.asarray(log_mass, dtype=np.float64).reshape(-1))
        nat.check(nat.lib().pf_debug_set_state(self._h, _ptr(s), None if L is None else _ptr(L),
                                               step), "pf_debug_set_state")

    def set_lineage(self, tags) -> None:
        t = np.ascontiguousarray(np.asarray(tags, dtype=np.int32).reshape(self.N))
        nat.check(nat.lib().pf_debug_set_lineage(self._h, _ptr(t)), "pf_debug_set_lineage")

    def force_next(self, anc=None, nex=None) -> None:
        """Make the next iteration use these ancestors ([N], slot within the
        PE, sorted within each PE) and/or N_ex ([F]) instead of its own
        (replay of another run's choices; test support)."""
        import torch
        keep = []
        ptrs = []
        for arr, n in ((anc, self.N), (nex, self.F)):
            if arr is None:
                ptrs.append(None)
                continue
            a = np.ascontiguousarray(np.asarray(arr, dtype=np.uint32).reshape(n))
            t = torch.from_numpy(a.view(np.int32)).cuda()
            keep.append(t)
            ptrs.append(ctypes.c_void_p(t.data_ptr()))
        self._forced = keep      # alive until the next iteration has run
        nat.check(nat.lib().pf_debug_force_next(self._h, ptrs[0], ptrs[1]), "pf_debug_force_next")

    def close(self) -> None:
        h = getattr(self, "_h", None)
        if h:
            nat.lib().pf_destroy(h)
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


# ------------------------------------------------------- device integer stages
def resample_q(Q, V) -> np.ndarray:
    """Systematic ancestors on the device: Q [B][n_p] uint32, V [B] uint32."""
    Q = np.ascontiguousarray(np.atleast_2d(np.asarray(Q, dtype=np.uint32)))
    V = np.ascontiguousarray(np.atleast_1d(np.asarray(V, dtype=np.uint32)))
    B, n_p = Q.shape
    anc = np.zeros((B, n_p), np.uint32)
    nat.check(nat.lib().pf_debug_resample_q(_ptr(Q), B, n_p, _ptr(V), _ptr(anc)),
              "pf_debug_resample_q")
    return anc


def nex(P, n_p: int, mode: int = nat.PF_MODE_ARNA, fixed_ratio: float = 0.1,
        initial_ratio: float = 0.1, cutoff: float = 0.99, first: bool = False) -> int:
    P = np.ascontiguousarray(np.asarray(P, dtype=np.uint32))
    out = ctypes.c_uint32()
    nat.check(nat.lib().pf_debug_nex(_ptr(P), len(P), n_p, mode, fixed_ratio, initial_ratio,
                                     cutoff, int(first), ctypes.byref(out)), "pf_debug_nex")
    return int(out.value)


def ring(seed: int, f: int, k: int, M: int, mode: int = nat.PF_MODE_ARNA,
         groups: int = 0) -> np.ndarray:
    pred = np.zeros(M, np.uint32)
    nat.check(nat.lib().pf_debug_ring(seed, f, k, M, mode, groups, _ptr(pred)), "pf_debug_ring")
    return pred


def philox(ctr, key) -> np.ndarray:
    c = np.ascontiguousarray(np.atleast_2d(np.asarray(ctr, dtype=np.uint32)))
    k = np.ascontiguousarray(np.asarray(key, dtype=np.uint32))
    out = np.zeros_like(c)
    nat.check(nat.lib().pf_debug_philox(_ptr(c), _ptr(k), c.shape[0], _ptr(out)),
              "pf_debug_philox")
    return out


class Batch:
    """Several Trackers advanced together (pf_batch_*): one launch per group
    of contexts sharing a kernel variant, optionally one HIP graph per run."""

    def __init__(self, trackers):
        self.trackers = list(trackers)
        arr = (ctypes.c_void_p * len(self.trackers))(*[t._h for t in self.trackers])
        h = ctypes.c_void_p()
        nat.check(nat.lib().pf_batch_create(arr, len(self.trackers), ctypes.byref(h)),
                  "pf_batch_create")
        self._h = h

    def run(self, frames, n_steps: int | None = None, graph: bool = False,
            no_alloc: bool = False) -> None:
        """frames[i]: the frames of tracker i (first axis = iteration).
        no_alloc: the entry point that allocates no device memory (argument
        table in the library's fixed per-GPU array; no graph)."""
        if no_alloc and graph:
            raise ValueError("the no-allocation run has no graph mode")
        if len(frames) != len(self.trackers):
            raise ValueError("one frame stack per tracker")
        n = min(f.shape[0] for f in frames) if n_steps is None else n_steps
        ptrs, strides = [], []
        for t, f in zip(self.trackers, frames):
            if f.shape[0] < n:
                raise ValueError("more steps than frames")
            stride = int(np.prod(f.shape[1:]))
            if stride != t.frame_numel():
                raise ValueError(f"frames hold {stride} values each, expected {t.frame_numel()}")
            ptrs.append(_dev_ptr(f, "frames").value)
            strides.append(stride)
        P = (ctypes.c_void_p * len(ptrs))(*ptrs)
        S = (ctypes.c_uint64 * len(strides))(*strides)
        if no_alloc:
            nat.check(nat.lib().pf_batch_run_noalloc(self._h, P, S, n), "pf_batch_run_noalloc")
        else:
            nat.check(nat.lib().pf_batch_run(self._h, P, S, n, 1 if graph else 0), "pf_batch_run")

    def close(self) -> None:
        h = getattr(self, "_h", None)
        if h:
            nat.lib().pf_batch_destroy(h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass
