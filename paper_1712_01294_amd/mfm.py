"""Thin ctypes binding of libmfm.so (include/mfm.h): argument marshalling only.

Every step of the pass runs in the HIP library; PyTorch only provides device
memory and the stream.  Loading fails loudly when the library is missing or
no GPU is present: there is no CPU fallback.
"""
from __future__ import annotations

import ctypes as C
import os
from dataclasses import dataclass

import torch

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libmfm.so")

FP64, MIXED = 0, 1
SCHEME_MFM, SCHEME_MFV = 0, 1   # mfm_scheme

STATUS = {0: "MFM_OK", -1: "MFM_E_INVALID", -2: "MFM_E_HIP", -3: "MFM_E_NOCONV", -4: "MFM_E_ILLCOND",
          -5: "MFM_E_MINIMAGE", -6: "MFM_E_CAPACITY", -7: "MFM_E_NONFINITE", -8: "MFM_E_STATE"}

EXPORTS = ("mfm_create", "mfm_destroy", "mfm_build_neighbours", "mfm_solve_h", "mfm_gradients",
           "mfm_hydro_fluxes", "mfm_hydro_pass", "mfm_step", "mfm_get_counters", "mfm_check",
           "mfm_copy_flux_lists", "mfm_max_ngb", "mfm_status_str", "mfm_last_error",
           "mfm_hydro_pass_adjoint", "mfm_step_adjoint", "mfm_tape_bytes", "mfm_step_taped",
           "mfm_step_adjoint_taped", "mfm_set_kernel_timing", "mfm_kernel_time",
           "mfm_hydro_pass_noalloc", "mfm_step_hier", "mfm_copy_levels", "mfm_unpermute",
           "mfm_limit_bins")

# kernels that mfm_kernel_time can report (mfm_kernel)
KERNELS = {"solve_h": 0, "gradients": 1, "hydro_fluxes": 2}


class Params(C.Structure):
    _fields_ = [("gamma", C.c_double), ("n_ngb", C.c_double), ("cfl", C.c_double),
                ("box", C.c_double * 3), ("periodic", C.c_int32 * 3), ("precision", C.c_int32),
                ("beta", C.c_double), ("cond_max", C.c_double), ("u_floor", C.c_double),
                ("h_maxit", C.c_int32), ("max_ngb", C.c_int32), ("tree_levels", C.c_int32),
                ("scheme", C.c_int32), ("limiter", C.c_int32), ("beta_min", C.c_double),
                ("cond_lo", C.c_double), ("cond_hi", C.c_double)]


_dp = C.POINTER(C.c_double)


class Particles(C.Structure):
    _fields_ = [("n", C.c_int64), ("x", _dp), ("y", _dp), ("z", _dp), ("m", _dp), ("vx", _dp),
                ("vy", _dp), ("vz", _dp), ("u", _dp), ("H", _dp), ("nk", _dp), ("V", _dp),
                ("B", _dp), ("rho", _dp), ("P", _dp), ("grad", _dp), ("alpha", _dp), ("dp", _dp),
                ("dE", _dp), ("vsig", _dp), ("id", C.POINTER(C.c_int64)), ("dm", _dp)]


class Counters(C.Structure):
    _fields_ = [(k, C.c_int64) for k in ("pairs", "list_entries", "list_max", "h_iters", "h_iters_max",
                                         "noconv", "minimage", "overflow", "illcond", "fallbacks",
                                         "clamps", "nonfinite", "floors", "first_bad")] + \
               [("cond_max_seen", C.c_double), ("h_rounds_max", C.c_int64), ("h_fallback", C.c_int64),
                ("h_rounds3", C.c_int64), ("gather_entries", C.c_int64), ("h_rescan", C.c_int64)]

    def as_dict(self):
        return {k: getattr(self, k) for k, _ in self._fields_}


class MFMError(RuntimeError):
    def __init__(self, status, msg):
        super().__init__(f"{STATUS.get(status, status)}: {msg}")
        self.status = status


_lib = None


def lib() -> C.CDLL:
    """Load libmfm.so; raise if it is missing (build it with paper_1712_01294_amd.build)."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise RuntimeError(f"{LIB_PATH} is not built: run python -m paper_1712_01294_amd.build")
        L = C.CDLL(LIB_PATH)
        vp = C.c_void_p
        L.mfm_create.argtypes = [C.POINTER(Params), C.c_int64, C.POINTER(vp)]
        L.mfm_destroy.argtypes = [vp]
        L.mfm_destroy.restype = None
        for f in ("mfm_build_neighbours", "mfm_solve_h", "mfm_gradients", "mfm_hydro_fluxes",
                  "mfm_hydro_pass", "mfm_unpermute"):
            getattr(L, f).argtypes = [vp, C.POINTER(Particles), vp]
        L.mfm_step.argtypes = [vp, C.POINTER(Particles), C.c_double, C.POINTER(C.c_double), vp]
        L.mfm_get_counters.argtypes = [vp, C.POINTER(Counters)]
        L.mfm_check.argtypes = [vp]
        L.mfm_copy_flux_lists.argtypes = [vp, vp, vp, vp]
        L.mfm_max_ngb.argtypes = [vp]
        L.mfm_max_ngb.restype = C.c_int32
        L.mfm_status_str.argtypes = [C.c_int]
        L.mfm_status_str.restype = C.c_char_p
        L.mfm_last_error.argtypes = [vp]
        L.mfm_last_error.restype = C.c_char_p
        L.mfm_hydro_pass_adjoint.argtypes = [vp, C.POINTER(Particles), vp, vp, vp, vp, vp, vp]
        L.mfm_step_adjoint.argtypes = [vp, C.POINTER(Particles), C.POINTER(Particles), C.c_double, vp, vp, vp,
                                       vp, vp, vp]
        L.mfm_tape_bytes.argtypes = [vp]
        L.mfm_tape_bytes.restype = C.c_int64
        L.mfm_step_taped.argtypes = [vp, C.POINTER(Particles), C.c_double, vp, vp]
        L.mfm_step_adjoint_taped.argtypes = [vp, C.POINTER(Particles), vp, C.c_double, vp, vp, vp, vp, vp, vp]
        L.mfm_set_kernel_timing.argtypes = [vp, C.c_int]
        L.mfm_kernel_time.argtypes = [vp, C.c_int, C.POINTER(C.c_double), C.POINTER(C.c_int64)]
        L.mfm_hydro_pass_noalloc.argtypes = [C.POINTER(Params), C.POINTER(Particles), C.POINTER(Counters), vp]
        L.mfm_step_hier.argtypes = [vp, C.POINTER(Particles), vp, C.c_int32, C.c_double, C.c_int32, vp]
        L.mfm_copy_levels.argtypes = [vp, vp, vp]
        L.mfm_limit_bins.argtypes = [vp, C.POINTER(Particles), vp, C.c_int32, C.POINTER(C.c_int64), vp]
        _lib = L
    return _lib


def _ptr(t):
    if t is None:
        return None
    if not t.is_cuda:
        raise ValueError("particle arrays must live on the GPU")
    if not t.is_contiguous():
        raise ValueError("particle arrays must be contiguous")
    return C.cast(C.c_void_p(t.data_ptr()), _dp)


def _stream(stream=None):
    s = torch.cuda.current_stream() if stream is None else stream
    return C.c_void_p(s.cuda_stream)


@dataclass
class Config:
    gamma: float
    box: tuple
    periodic: tuple = (1, 1, 1)
    n_ngb: float = 32.0
    cfl: float = 0.25
    precision: int = FP64
    beta: float = 1.0
    cond_max: float = 1.0e6
    u_floor: float = 0.0
    h_maxit: int = 64
    max_ngb: int = 256
    tree_levels: int = 0
    scheme: int = SCHEME_MFM
    limiter: int = 0          # 1: pairwise face limiter (R23) and condition-adaptive beta (R24)
    beta_min: float = 1.0
    cond_lo: float = 10.0
    cond_hi: float = 1000.0

    def c(self) -> Params:
        p = Params()
        p.gamma = self.gamma
        p.n_ngb = self.n_ngb
        p.cfl = self.cfl
        for a in range(3):
            p.box[a] = self.box[a]
            p.periodic[a] = int(self.periodic[a])
        p.precision = int(self.precision)
        p.beta = self.beta
        p.cond_max = self.cond_max
        p.u_floor = self.u_floor
        p.h_maxit = self.h_maxit
        p.max_ngb = self.max_ngb
        p.tree_levels = self.tree_levels
        p.scheme = int(self.scheme)
        p.limiter = int(self.limiter)
        p.beta_min = self.beta_min
        p.cond_lo = self.cond_lo
        p.cond_hi = self.cond_hi
        return p


class State:
    """Device-resident SoA particle arrays (float64) in the layout of mfm_particles."""

    INPUTS = ("x", "y", "z", "m", "vx", "vy", "vz", "u")

    def __init__(self, n: int, device="cuda", alpha: bool = False, ids: bool = True, dm: bool = False,
                 zero: bool = True):
        """zero=False leaves the arrays uninitialised (for states whose every
        array is written before it is read, such as checkpoint copies)."""
        f = dict(dtype=torch.float64, device=device)
        new = torch.zeros if zero else torch.empty
        self.n = n
        for k in self.INPUTS + ("H", "nk", "V", "rho", "P", "dE", "vsig"):
            setattr(self, k, new(n, **f))
        self.B = new(6, n, **f)
        self.grad = new(15, n, **f)
        self.dp = new(3, n, **f)
        self.alpha = new(5, n, **f) if alpha else None
        self.id = torch.arange(n, dtype=torch.int64, device=device) if ids else None
        self.dm = new(n, **f) if dm else None

    @classmethod
    def from_arrays(cls, arrays: dict, device="cuda", **kw) -> "State":
        n = int(arrays["x"].shape[0])
        st = cls(n, device=device, **kw)
        for k in cls.INPUTS:
            getattr(st, k).copy_(torch.as_tensor(arrays[k], dtype=torch.float64))
        return st

    def struct(self) -> Particles:
        p = Particles()
        p.n = self.n
        for k in ("x", "y", "z", "m", "vx", "vy", "vz", "u", "H", "nk", "V", "B", "rho", "P", "grad",
                  "alpha", "dp", "dE", "vsig", "dm"):
            setattr(p, k, _ptr(getattr(self, k)))
        p.id = C.cast(C.c_void_p(self.id.data_ptr()), C.POINTER(C.c_int64)) if self.id is not None else None
        return p


class Context:
    """One library context (scratch for up to `capacity` particles)."""

    def __init__(self, cfg: Config, capacity: int):
        self.cfg = cfg
        self._L = lib()
        h = C.c_void_p()
        rc = self._L.mfm_create(C.byref(cfg.c()), C.c_int64(capacity), C.byref(h))
        if rc != 0:
            raise MFMError(rc, "mfm_create failed (bad parameters or out of device memory)")
        self.h = h
        self.capacity = capacity

    def close(self):
        if self.h:
            self._L.mfm_destroy(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def _rc(self, rc):
        if rc != 0:
            raise MFMError(rc, self._L.mfm_last_error(self.h).decode())

    def _call(self, name, st: State, stream=None):
        p = st.struct()
        self._rc(getattr(self._L, name)(self.h, C.byref(p), _stream(stream)))

    def build_neighbours(self, st: State, stream=None):
        self._call("mfm_build_neighbours", st, stream)

    def unpermute(self, st: State, stream=None):
        """Move every array of st back to the order the particles were given in
        (particle k to position st.id[k]); afterwards st.id is 0 .. n-1.  The
        next pass needs build_neighbours first."""
        self._call("mfm_unpermute", st, stream)

    def solve_h(self, st: State, stream=None):
        self._call("mfm_solve_h", st, stream)

    def gradients(self, st: State, stream=None):
        self._call("mfm_gradients", st, stream)

    def hydro_fluxes(self, st: State, stream=None):
        self._call("mfm_hydro_fluxes", st, stream)

    def hydro_pass(self, st: State, stream=None):
        self._call("mfm_hydro_pass", st, stream)

    def step(self, st: State, dt: float = 0.0, stream=None) -> float:
        p = st.struct()
        used = C.c_double(0.0)
        self._rc(self._L.mfm_step(self.h, C.byref(p), C.c_double(dt), C.byref(used), _stream(stream)))
        return used.value

    def limit_bins(self, st: State, bins, max_bin: int, stream=None) -> int:
        """The neighbour time-step limiter (mfm_limit_bins): raises bins (int64
        device tensor, n, st's current order) in place so that flux neighbours
        lie at most one bin apart; returns the number of raises."""
        if bins.dtype != torch.int64 or not bins.is_cuda or not bins.is_contiguous():
            raise ValueError("bins must be a contiguous int64 device tensor")
        p = st.struct()
        raised = C.c_int64(0)
        self._rc(self._L.mfm_limit_bins(self.h, C.byref(p), C.c_void_p(bins.data_ptr()), C.c_int32(max_bin),
                                        C.byref(raised), _stream(stream)))
        return int(raised.value)

    def step_hier(self, st: State, bins, max_bin: int, T: float, rebin: bool = False, active: bool = False,
                  stream=None):
        """One system step of length T with hierarchical power-of-two steps
        (mfm_step_hier); bins (int64 device tensor, n) is reordered with st.
        rebin: MFM_HIER_REBIN; active: MFM_HIER_ACTIVE (active subsets)."""
        if bins.dtype != torch.int64 or not bins.is_cuda or not bins.is_contiguous():
            raise ValueError("bins must be a contiguous int64 device tensor")
        p = st.struct()
        self._rc(self._L.mfm_step_hier(self.h, C.byref(p), C.c_void_p(bins.data_ptr()), C.c_int32(max_bin),
                                       C.c_double(T), C.c_int32((HIER_REBIN if rebin else 0) | (HIER_ACTIVE if active else 0)),
                                       _stream(stream)))

    def levels(self, n: int, nlev: int, stream=None):
        """The per-level rates of the last hierarchical step's last boundary,
        (nlev, 4, n): dp x, y, z and dE per level, in the current order."""
        out = torch.empty(nlev, 4, n, dtype=torch.float64, device="cuda")
        self._rc(self._L.mfm_copy_levels(self.h, C.c_void_p(out.data_ptr()), _stream(stream)))
        return out

    def pass_adjoint(self, st: State, adj_dp, adj_dE, stream=None):
        """(dF/d(x, v, u))^T (adj_dp, adj_dE) for the pass last run on st;
        returns adj_x (3, n), adj_v (3, n), adj_u (n) in st's order."""
        n = st.n
        f = dict(dtype=torch.float64, device="cuda")
        ax, av, au = torch.empty(3, n, **f), torch.empty(3, n, **f), torch.empty(n, **f)
        p = st.struct()
        v = lambda t: C.c_void_p(t.data_ptr())
        self._rc(self._L.mfm_hydro_pass_adjoint(self.h, C.byref(p), v(adj_dp.contiguous()),
                                                v(adj_dE.contiguous()), v(ax), v(av), v(au), _stream(stream)))
        return ax, av, au

    def step_adjoint(self, ckpt: State, work: State, dt: float, ax, av, au, ap, ae, stream=None):
        """In place: adjoints of the state after one fixed-dt step (in the order the
        step produced) -> adjoints of the checkpointed state (in its order)."""
        pc, pw = ckpt.struct(), work.struct()
        v = lambda t: C.c_void_p(t.data_ptr())
        self._rc(self._L.mfm_step_adjoint(self.h, C.byref(pc), C.byref(pw), C.c_double(dt), v(ax), v(av), v(au),
                                          v(ap), v(ae), _stream(stream)))

    def tape_bytes(self) -> int:
        return int(self._L.mfm_tape_bytes(self.h))

    def step_taped(self, st: State, dt: float, tape, stream=None):
        """mfm_step with a fixed dt that also records the step's tape (a device
        uint8 tensor of tape_bytes() bytes)."""
        p = st.struct()
        self._rc(self._L.mfm_step_taped(self.h, C.byref(p), C.c_double(dt), C.c_void_p(tape.data_ptr()),
                                        _stream(stream)))

    def step_adjoint_taped(self, ckpt: State, tape, dt: float, ax, av, au, ap, ae, stream=None):
        """step_adjoint reading the step from its tape instead of recomputing it."""
        pc = ckpt.struct()
        v = lambda t: C.c_void_p(t.data_ptr())
        self._rc(self._L.mfm_step_adjoint_taped(self.h, C.byref(pc), v(tape), C.c_double(dt), v(ax), v(av), v(au),
                                                v(ap), v(ae), _stream(stream)))

    def counters(self) -> dict:
        c = Counters()
        self._rc(self._L.mfm_get_counters(self.h, C.byref(c)))
        return c.as_dict()

    def set_kernel_timing(self, enable: bool = True):
        """Bracket every launch of the three pass kernels with HIP events on the
        call's stream (enabling also zeroes the totals)."""
        self._rc(self._L.mfm_set_kernel_timing(self.h, 1 if enable else 0))

    def kernel_time(self, kernel: str):
        """(total milliseconds, launches) of one pass kernel since timing was enabled."""
        ms, k = C.c_double(), C.c_int64()
        self._rc(self._L.mfm_kernel_time(self.h, KERNELS[kernel], C.byref(ms), C.byref(k)))
        return ms.value, k.value

    def check(self, allow_illcond: bool = False):
        """Raise on device-side conditions.  With allow_illcond, ill-conditioned
        gradient matrices (a reported count on strongly clustered sets) pass."""
        rc = self._L.mfm_check(self.h)
        if rc == -4 and allow_illcond:
            return
        self._rc(rc)

    def flux_lists(self, n: int, stream=None):
        mx = int(self._L.mfm_max_ngb(self.h))
        counts = torch.zeros(n, dtype=torch.int32, device="cuda")
        lst = torch.zeros(mx, n, dtype=torch.int32, device="cuda")
        self._rc(self._L.mfm_copy_flux_lists(self.h, C.c_void_p(counts.data_ptr()),
                                             C.c_void_p(lst.data_ptr()), _stream(stream)))
        return counts, lst


HIER_REBIN, HIER_ACTIVE = 1, 2   # mfm_step_hier flags (MFM_HIER_REBIN, MFM_HIER_ACTIVE)


NOALLOC_MAX_N = 8192   # particles per mfm_hydro_pass_noalloc call


def hydro_pass_noalloc(cfg: Config, st: State, counters: bool = True, stream=None):
    """mfm_hydro_pass_noalloc: neighbours and the whole pass without a context or
    any device allocation (st is reordered in place).  With counters the call
    synchronises and returns the counter dict (raising on device-side errors
    as Context.check does, ill-conditioned gradient matrices included); without,
    it only queues the work and returns None."""
    L = lib()
    p = st.struct()
    out = Counters() if counters else None
    rc = L.mfm_hydro_pass_noalloc(C.byref(cfg.c()), C.byref(p), C.byref(out) if counters else None,
                                  _stream(stream))
    if rc != 0:
        raise MFMError(rc, "mfm_hydro_pass_noalloc failed")
    return out.as_dict() if counters else None


def config_of(w, precision=FP64, **kw) -> Config:
    """Context configuration for a workload from ``workloads``."""
    u_floor = kw.pop("u_floor", 1e-10 * float(sum(w.u) / len(w.u)))
    return Config(gamma=w.gamma, box=tuple(w.box), periodic=tuple(w.periodic), n_ngb=w.n_ngb,
                  cfl=w.cfl, precision=precision, u_floor=u_floor, **kw)
