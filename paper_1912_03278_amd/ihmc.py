"""Python binding of the MI355X HMC library (include/ihmc.h).

Argument marshalling only: every step of the method runs in the HIP kernels of
``libihmc.so``.  PyTorch supplies device memory (the library's arena is one
block from torch's caching allocator) and nothing else.  There is no CPU
fallback: if the library or a GPU is missing, every call raises.
"""
from __future__ import annotations

import ctypes as C
import os
from dataclasses import dataclass, field

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.environ.get("IHMC_LIB", os.path.join(HERE, "libihmc.so"))

IHMC_OK = 0
STATUS = {-1: "IHMC_E_INVAL", -2: "IHMC_E_NOMEM", -3: "IHMC_E_AGAIN", -4: "IHMC_E_DEVICE",
          -5: "IHMC_E_CANCELLED", -6: "IHMC_E_UNSUPPORTED"}
F32, F64 = 4, 8
LEAPFROG, OMELYAN = 0, 1
FORM_PSI, FORM_PHI = 0, 1  # the substituted field (the hot path) / the inverse formulation (A/B baseline)
FORM_SHIFTED = 2  # the substitution phi = sqrt(J') Kt psi: h' inside the log cosh
FIRST, MIDDLE, LAST, PAIR = 0, 1, 2, 5  # pass kinds of Chains.time_pass
TAG_INIT, TAG_MOM, TAG_ACC, TAG_FLIP = 1, 2, 3, 4

EXPORTS = (
    "ihmc_ctx_create", "ihmc_ctx_destroy", "ihmc_ctx_stream", "ihmc_ctx_sync", "ihmc_ctx_memory",
    "ihmc_last_error", "ihmc_chains_create", "ihmc_chains_advance", "ihmc_chains_result",
    "ihmc_chains_destroy", "ihmc_run_lattice", "ihmc_run_batch", "ihmc_force", "ihmc_action",
    "ihmc_integrate", "ihmc_philox_normals", "ihmc_philox_words", "ihmc_chains_groups",
    "ihmc_chains_time_pass", "ihmc_chains_group_info", "ihmc_copy_bandwidth", "ihmc_dense_create",
    "ihmc_dense_advance", "ihmc_dense_result", "ihmc_dense_info", "ihmc_dense_time", "ihmc_dense_destroy",
    "ihmc_run_dense", "ihmc_dense_force", "ihmc_min_eig", "ihmc_server_create", "ihmc_server_destroy",
    "ihmc_submit", "ihmc_poll", "ihmc_wait", "ihmc_fetch", "ihmc_cancel", "ihmc_server_stats",
    "ihmc_tile_shape", "ihmc_tune", "ihmc_tune_lookup", "ihmc_tune_pin", "ihmc_tune_save", "ihmc_tune_load",
    "ihmc_tune_check", "ihmc_chains_checkpoint", "ihmc_chains_restore", "ihmc_dense_checkpoint",
    "ihmc_dense_restore", "ihmc_ctx_set_resident", "ihmc_ctx_set_step_fusion", "ihmc_hamiltonian",
    "ihmc_plan_events", "ihmc_fixed_point", "ihmc_chains_group_chains", "ihmc_checkpoint", "ihmc_restore",
    "ihmc_request_info", "ihmc_force_noalloc", "ihmc_mh_run", "ihmc_dense_mh_run",
)
TUNE_RULE, TUNE_MEASURED, TUNE_PINNED = 0, 1, 2
REQ_QUEUED, REQ_RUNNING, REQ_DONE, REQ_CANCELLED, REQ_FAILED = 0, 1, 2, 3, 4


class IhmcError(RuntimeError):
    def __init__(self, code, msg):
        super().__init__(f"{STATUS.get(code, code)}: {msg}")
        self.code = code


class _Lattice(C.Structure):
    _fields_ = [("ndim", C.c_int32), ("L", C.c_int32 * 3), ("J", C.c_double), ("beta", C.c_double),
                ("C", C.c_double), ("h", C.POINTER(C.c_double)), ("h_len", C.c_int64)]


class _Dense(C.Structure):
    _fields_ = [("N", C.c_int64), ("K", C.POINTER(C.c_double)), ("J", C.c_double), ("beta", C.c_double),
                ("C", C.c_double), ("h", C.POINTER(C.c_double)), ("h_len", C.c_int64)]


class _Run(C.Structure):
    _fields_ = [("n_md", C.c_int32), ("n_traj", C.c_int32), ("traj_len", C.c_double),
                ("integrator", C.c_int32), ("flip_every", C.c_int32), ("precision", C.c_int32),
                ("n_therm", C.c_int32), ("seed", C.c_uint64), ("chain_id", C.c_uint64),
                ("psi0", C.POINTER(C.c_double)), ("replay_accept", C.POINTER(C.c_uint8)),
                ("form", C.c_int32), ("reserved", C.c_int32)]


_DP = C.POINTER(C.c_double)
_U8 = C.POINTER(C.c_uint8)


class _Result(C.Structure):
    _fields_ = [("dH", _DP), ("H_old", _DP), ("H_new", _DP), ("m", _DP), ("abs_m", _DP), ("m2c", _DP),
                ("beta_eps", _DP), ("accepted", _U8), ("flipped", _U8), ("psi_final", _DP),
                ("acceptance", C.c_double), ("mean_exp_minus_dH", C.c_double),
                ("n_nonfinite", C.c_int64), ("n_traj_done", C.c_int64), ("cg_iterations", C.c_int64)]


ALLOC_FN = C.CFUNCTYPE(C.c_void_p, C.c_uint64, C.c_void_p)
FREE_FN = C.CFUNCTYPE(None, C.c_void_p, C.c_void_p)

_lib = None


def load():
    """Load libihmc.so (built by paper_1912_03278_amd.build); raise if it is missing."""
    global _lib
    if _lib is not None:
        return _lib
    # PyTorch ships its own HIP runtime under the same soname; loading torch first
    # makes the library bind to that one runtime instead of a second copy.
    try:
        import torch  # noqa: F401
    except ImportError:
        pass
    if not os.path.exists(LIB_PATH):
        raise ImportError(f"{LIB_PATH} is missing: build it with `python -m paper_1912_03278_amd.build`")
    L = C.CDLL(LIB_PATH)
    vp, pp = C.c_void_p, C.POINTER(C.c_void_p)
    L.ihmc_ctx_create.argtypes = [C.c_int32, C.c_uint64, ALLOC_FN, FREE_FN, vp, pp]
    L.ihmc_ctx_destroy.argtypes = [vp]
    L.ihmc_ctx_destroy.restype = None
    L.ihmc_ctx_stream.argtypes = [vp]
    L.ihmc_ctx_stream.restype = vp
    L.ihmc_ctx_sync.argtypes = [vp]
    L.ihmc_ctx_memory.argtypes = [vp, C.POINTER(C.c_uint64), C.POINTER(C.c_uint64)]
    L.ihmc_ctx_set_resident.argtypes = [vp, C.c_int64, C.POINTER(C.c_int64), C.POINTER(C.c_int64)]
    L.ihmc_ctx_set_step_fusion.argtypes = [vp, C.c_int32]
    L.ihmc_last_error.restype = C.c_char_p
    L.ihmc_chains_create.argtypes = [vp, C.c_int32, C.POINTER(_Lattice), C.POINTER(_Run), pp]
    L.ihmc_chains_advance.argtypes = [vp, C.c_int32]
    L.ihmc_chains_result.argtypes = [vp, C.c_int32, C.POINTER(_Result)]
    L.ihmc_chains_destroy.argtypes = [vp]
    L.ihmc_chains_checkpoint.argtypes = [vp, C.c_int32, vp, C.POINTER(C.c_uint64)]
    L.ihmc_chains_restore.argtypes = [vp, C.c_int32, vp, C.c_uint64]
    L.ihmc_dense_checkpoint.argtypes = [vp, C.c_int32, vp, C.POINTER(C.c_uint64)]
    L.ihmc_dense_restore.argtypes = [vp, C.c_int32, vp, C.c_uint64]
    L.ihmc_run_lattice.argtypes = [vp, C.POINTER(_Lattice), C.POINTER(_Run), C.POINTER(_Result)]
    L.ihmc_run_batch.argtypes = [vp, C.c_int32, C.POINTER(_Lattice), C.POINTER(_Run), C.POINTER(_Result)]
    L.ihmc_force.argtypes = [vp, C.POINTER(_Lattice), C.c_int32, _DP, _DP]
    L.ihmc_force_noalloc.argtypes = [vp, C.POINTER(_Lattice), C.c_int32, vp, vp, vp]
    i8p = C.POINTER(C.c_int8)
    L.ihmc_mh_run.argtypes = [vp, C.POINTER(_Lattice), C.c_int32, C.c_uint64, C.c_uint64, i8p, _DP, _DP, i8p, _DP]
    L.ihmc_dense_mh_run.argtypes = [vp, C.POINTER(_Dense), C.c_int32, C.c_int32, C.c_uint64, C.c_uint64, i8p, _DP,
                                    _DP, i8p, _DP, _DP]
    L.ihmc_action.argtypes = [vp, C.POINTER(_Lattice), C.c_int32, _DP, _DP]
    L.ihmc_integrate.argtypes = [vp, C.POINTER(_Lattice), C.POINTER(_Run), _DP, _DP]
    L.ihmc_philox_normals.argtypes = [vp, C.c_uint64, C.c_uint64, C.c_uint32, C.c_uint32, C.c_int32, C.c_int64,
                                      _DP]
    L.ihmc_hamiltonian.argtypes = [vp, C.POINTER(_Lattice), C.c_int32, _DP, _DP, _DP]
    L.ihmc_plan_events.argtypes = [C.c_int32, C.POINTER(_Lattice), C.POINTER(_Run), C.c_int32, C.c_int64,
                                   C.POINTER(C.c_int64), C.POINTER(C.c_int64)]
    L.ihmc_fixed_point.argtypes = [C.c_int64, _DP, C.POINTER(C.c_uint64), C.POINTER(C.c_int32)]
    L.ihmc_philox_words.argtypes = [vp, C.c_int64, C.POINTER(C.c_uint32), C.POINTER(C.c_uint32),
                                    C.POINTER(C.c_uint32)]
    L.ihmc_chains_groups.argtypes = [vp, C.POINTER(C.c_int32)]
    L.ihmc_chains_group_info.argtypes = [vp, C.c_int32, C.POINTER(C.c_int64)]
    L.ihmc_chains_group_chains.argtypes = [vp, C.c_int32, C.POINTER(C.c_int32)]
    L.ihmc_chains_time_pass.argtypes = [vp, C.c_int32, C.c_int32, C.c_int32, C.POINTER(C.c_double),
                                        C.POINTER(C.c_int64), C.POINTER(C.c_int32), C.POINTER(C.c_int32)]
    L.ihmc_copy_bandwidth.argtypes = [vp, C.c_uint64, C.c_int32, C.POINTER(C.c_double)]
    L.ihmc_dense_create.argtypes = [vp, C.POINTER(_Dense), C.c_int32, C.POINTER(_Run), C.c_int32, pp]
    L.ihmc_dense_advance.argtypes = [vp, C.c_int32]
    L.ihmc_dense_result.argtypes = [vp, C.c_int32, C.POINTER(_Result)]
    L.ihmc_dense_info.argtypes = [vp, _DP]
    L.ihmc_dense_time.argtypes = [vp, C.c_int32, C.c_int32, C.POINTER(C.c_double), C.POINTER(C.c_int64)]
    L.ihmc_dense_destroy.argtypes = [vp]
    L.ihmc_run_dense.argtypes = [vp, C.POINTER(_Dense), C.c_int32, C.POINTER(_Run), C.c_int32,
                                 C.POINTER(_Result)]
    L.ihmc_dense_force.argtypes = [vp, C.POINTER(_Dense), C.c_int32, _DP, C.c_int32, _DP]
    L.ihmc_min_eig.argtypes = [vp, _DP, C.c_int64, _DP, _DP, C.POINTER(C.c_int32)]
    L.ihmc_server_create.argtypes = [vp, C.c_uint64, C.c_int32, pp]
    L.ihmc_server_destroy.argtypes = [vp]
    L.ihmc_submit.argtypes = [vp, C.POINTER(_Lattice), C.POINTER(_Run), C.POINTER(C.c_uint64)]
    L.ihmc_poll.argtypes = [vp, C.c_uint64, C.POINTER(C.c_int32)]
    L.ihmc_wait.argtypes = [vp, C.c_uint64, C.c_double, C.POINTER(C.c_int32)]
    L.ihmc_fetch.argtypes = [vp, C.c_uint64, C.POINTER(_Result), _DP]
    L.ihmc_cancel.argtypes = [vp, C.c_uint64]
    L.ihmc_server_stats.argtypes = [vp, _DP]
    L.ihmc_checkpoint.argtypes = [vp, C.c_uint64, vp, C.POINTER(C.c_uint64)]
    L.ihmc_restore.argtypes = [vp, vp, C.c_uint64, C.POINTER(C.c_uint64)]
    L.ihmc_request_info.argtypes = [vp, C.c_uint64, C.POINTER(C.c_int64)]
    i32p = C.POINTER(C.c_int32)
    L.ihmc_tile_shape.argtypes = [C.c_int32, C.c_int32, i32p, i32p]
    L.ihmc_tune.argtypes = [vp, C.c_int32, C.POINTER(_Lattice), i32p, C.c_int64, C.c_int32, C.c_int32, i32p]
    L.ihmc_tune_lookup.argtypes = [vp, C.POINTER(_Lattice), C.c_int32, i32p, i32p, _DP]
    L.ihmc_tune_pin.argtypes = [vp, C.POINTER(_Lattice), C.c_int32, C.c_int32]
    L.ihmc_tune_save.argtypes = [vp, C.c_char_p]
    L.ihmc_tune_load.argtypes = [vp, C.c_char_p]
    L.ihmc_tune_check.argtypes = [C.c_char_p, i32p]
    _lib = L
    return L


def _check(rc):
    if rc != IHMC_OK:
        raise IhmcError(rc, load().ihmc_last_error().decode(errors="replace"))


def tile_shape(ndim, cls):
    """(x, y, z) extent of tile class `cls` of the lattice passes in dimension ndim."""
    out = (C.c_int32 * 3)()
    _check(load().ihmc_tile_shape(int(ndim), int(cls), out, None))
    return tuple(out)


def tile_class_count(ndim):
    n = C.c_int32()
    _check(load().ihmc_tile_shape(int(ndim), 0, None, C.byref(n)))
    return n.value


def check_tuning(path):
    """Parse a saved tile-class table (no GPU needed); returns its number of entries."""
    n = C.c_int32()
    _check(load().ihmc_tune_check(os.fsencode(path), C.byref(n)))
    return n.value


def _f64(a):
    return None if a is None else np.ascontiguousarray(a, dtype=np.float64)


def plan_events(lats, runs, fuse_steps=True, resident_sites=-1):
    """(events one round of the chain set's launch plan takes, events the set
    reserves for it), from a dry run on the host (no GPU needed)."""
    keep = []
    n = len(lats)
    la = (_Lattice * n)(*[l._c(keep) for l in lats])
    ra = (_Run * n)(*[r._c(keep) for r in runs])
    taken, reserved = C.c_int64(), C.c_int64()
    _check(load().ihmc_plan_events(n, la, ra, 1 if fuse_steps else 0, int(resident_sites), C.byref(taken),
                                   C.byref(reserved)))
    return taken.value, reserved.value


def fixed_point(x):
    """The library's fixed-point form of single action changes (host-only):
    (signed 128-bit integers round(x 2^64) as Python ints, ok flags)."""
    x = np.ascontiguousarray(np.atleast_1d(x), dtype=np.float64)
    out = np.zeros(2 * x.size, dtype=np.uint64)
    ok = np.zeros(x.size, dtype=np.int32)
    _check(load().ihmc_fixed_point(x.size, _dp(x), out.ctypes.data_as(C.POINTER(C.c_uint64)),
                                   ok.ctypes.data_as(C.POINTER(C.c_int32))))
    vals = []
    for k in range(x.size):
        v = int(out[2 * k]) | (int(out[2 * k + 1]) << 64)
        vals.append(v - (1 << 128) if v >> 127 else v)
    return vals, ok.astype(bool)


def _dp(a):
    return None if a is None else a.ctypes.data_as(_DP)


@dataclass
class Lattice:
    """Periodic 2D/3D nearest-neighbour lattice (Sec. 2): J' = beta J, Kt = K + C 1."""
    L: tuple
    beta: float
    C: float
    J: float = 1.0
    h: object = None  # None, a scalar, or one value per site

    @property
    def N(self):
        return int(np.prod(self.L))

    def _c(self, keep):
        s = _Lattice()
        s.ndim = len(self.L)
        for i in range(3):
            s.L[i] = int(self.L[i]) if i < len(self.L) else 1
        s.J, s.beta, s.C = float(self.J), float(self.beta), float(self.C)
        h = None if self.h is None else _f64(np.atleast_1d(self.h))
        keep.append(h)
        s.h = _dp(h)
        s.h_len = 0 if h is None else h.size
        return s


@dataclass
class Dense:
    """Explicit symmetric coupling matrix K (the model's couplings are J K), Kt = K + C 1.
    C < 0 selects the shift from the lowest Ritz value of K (FP64 Lanczos)."""
    K: object
    beta: float
    C: float = -1.0
    J: float = 1.0
    h: object = None  # None, a scalar, or one value per site

    def __post_init__(self):
        self.K = np.ascontiguousarray(self.K, dtype=np.float64)
        if self.K.ndim != 2 or self.K.shape[0] != self.K.shape[1]:
            raise ValueError("K must be a square matrix")

    @property
    def N(self):
        return int(self.K.shape[0])

    def _c(self, keep):
        s = _Dense()
        s.N = self.N
        keep.append(self.K)
        s.K = _dp(self.K)
        s.J, s.beta, s.C = float(self.J), float(self.beta), float(self.C)
        h = None if self.h is None else _f64(np.atleast_1d(self.h))
        keep.append(h)
        s.h = _dp(h)
        s.h_len = 0 if h is None else h.size
        return s


@dataclass
class Run:
    """Chain parameters (Sec. 3)."""
    n_md: int
    n_traj: int
    traj_len: float = 1.0
    integrator: int = LEAPFROG
    flip_every: int = 0
    precision: int = F32
    seed: int = 0
    chain_id: int = 0
    psi0: object = None
    replay_accept: object = None
    n_therm: int = 0
    form: int = FORM_PSI

    def _c(self, keep):
        s = _Run()
        s.n_md, s.n_traj, s.traj_len = int(self.n_md), int(self.n_traj), float(self.traj_len)
        s.integrator, s.flip_every, s.precision = int(self.integrator), int(self.flip_every), int(self.precision)
        s.n_therm = int(self.n_therm)
        s.form = int(self.form)
        s.seed, s.chain_id = int(self.seed), int(self.chain_id)
        p0 = _f64(self.psi0)
        keep.append(p0)
        s.psi0 = _dp(p0)
        ra = None if self.replay_accept is None else np.ascontiguousarray(self.replay_accept, dtype=np.uint8)
        keep.append(ra)
        s.replay_accept = None if ra is None else ra.ctypes.data_as(_U8)
        return s


SERIES = ("dH", "H_old", "H_new", "m", "abs_m", "m2c", "beta_eps")


def _result_struct(n_traj, N, want_psi=True):
    arrays = {k: np.zeros(n_traj) for k in SERIES}
    arrays["accepted"] = np.zeros(n_traj, dtype=np.uint8)
    arrays["flipped"] = np.zeros(n_traj, dtype=np.uint8)
    if want_psi:
        arrays["psi_final"] = np.zeros(N)
    r = _Result()
    for k, v in arrays.items():
        setattr(r, k, v.ctypes.data_as(_U8 if v.dtype == np.uint8 else _DP))
    return r, arrays


def _result_dict(r, arrays):
    out = dict(arrays)
    out.update(acceptance=r.acceptance, mean_exp_minus_dH=r.mean_exp_minus_dH,
               n_nonfinite=int(r.n_nonfinite), n_traj_done=int(r.n_traj_done),
               cg_iterations=int(r.cg_iterations))
    return out


class Context:
    """A device context: HIP stream plus an arena of device memory from torch."""

    def __init__(self, device=0, arena_bytes=1 << 30, use_torch=True, resident=-1, fuse_steps=True):
        L = load()
        self._keep = []
        if use_torch:
            import torch
            if not torch.cuda.is_available():
                raise RuntimeError("no GPU visible to torch")
            dev = int(device)

            def _alloc(nbytes, user):
                return int(torch.cuda.caching_allocator_alloc(int(nbytes), device=dev))

            def _free(ptr, user):
                # at interpreter shutdown torch may already be torn down
                tc = getattr(torch, "cuda", None)
                if tc is not None:
                    tc.caching_allocator_delete(int(ptr))

            af, ff = ALLOC_FN(_alloc), FREE_FN(_free)
        else:
            af, ff = ALLOC_FN(), FREE_FN()
        self._fns = (af, ff)
        h = C.c_void_p()
        _check(L.ihmc_ctx_create(int(device), int(arena_bytes), af, ff, None, C.byref(h)))
        self.h = h
        if resident != -1:
            self.set_resident(resident)
        if not fuse_steps:
            self.set_step_fusion(False)

    def set_resident(self, max_sites=-1):
        """Chains created afterwards with at most max_sites sites (and small enough
        for one workgroup's LDS) run LDS-resident whole trajectories; -1 admits
        every chain that fits, 0 none.  Returns the largest FP32 and FP64 chains
        that fit (without a per-site field)."""
        f32, f64 = C.c_int64(), C.c_int64()
        _check(load().ihmc_ctx_set_resident(self.h, int(max_sites), C.byref(f32), C.byref(f64)))
        return f32.value, f64.value

    def set_step_fusion(self, on=True):
        """2D chains on the tiled passes run their middle steps two per launch
        (bit-identical results); applies to chain sets created afterwards."""
        _check(load().ihmc_ctx_set_step_fusion(self.h, 1 if on else 0))

    def close(self):
        if getattr(self, "h", None):
            load().ihmc_ctx_destroy(self.h)
            self.h = None

    def __enter__(self):
        return self

    def __exit__(self, *a):
        self.close()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    @property
    def stream(self):
        return load().ihmc_ctx_stream(self.h)

    def sync(self):
        _check(load().ihmc_ctx_sync(self.h))

    def memory(self):
        u, t = C.c_uint64(), C.c_uint64()
        _check(load().ihmc_ctx_memory(self.h, C.byref(u), C.byref(t)))
        return u.value, t.value

    # ---- tile autotuner
    def tune(self, lats, precision=F32, sites=0, reps=0, force=False):
        """Time every tile class on each distinct lattice shape and keep the fastest
        for chains created afterwards; returns the number of shapes measured.
        `sites`: working set of the timed launches (0: the total sites of `lats`)."""
        keep = []
        n = len(lats)
        prec = [precision] * n if isinstance(precision, int) else list(precision)
        la = (_Lattice * n)(*[l._c(keep) for l in lats])
        pa = (C.c_int32 * n)(*prec)
        got = C.c_int32()
        _check(load().ihmc_tune(self.h, n, la, pa, int(sites), int(reps), 1 if force else 0, C.byref(got)))
        return got.value

    def tile_class(self, lat: Lattice, precision=F32):
        """{'cls', 'source', 'ns_per_site'} of the tile class chains of `lat` take here."""
        keep = []
        s = lat._c(keep)
        cls, src = C.c_int32(), C.c_int32()
        ns = (C.c_double * 4)()
        _check(load().ihmc_tune_lookup(self.h, C.byref(s), int(precision), C.byref(cls), C.byref(src), ns))
        return {"cls": cls.value, "source": src.value, "ns_per_site": list(ns)}

    def pin_tile(self, lat: Lattice, cls, precision=F32):
        """Force tile class `cls` for chains of `lat` (cls < 0: back to the built-in rule)."""
        keep = []
        s = lat._c(keep)
        _check(load().ihmc_tune_pin(self.h, C.byref(s), int(precision), int(cls)))

    def save_tuning(self, path):
        _check(load().ihmc_tune_save(self.h, os.fsencode(path)))

    def load_tuning(self, path):
        _check(load().ihmc_tune_load(self.h, os.fsencode(path)))

    # ---- whole runs
    def run_lattice(self, lat: Lattice, run: Run, want_psi=True):
        return self.run_batch([lat], [run], want_psi)[0]

    def run_batch(self, lats, runs, want_psi=True):
        keep = []
        n = len(lats)
        la = (_Lattice * n)(*[l._c(keep) for l in lats])
        ra = (_Run * n)(*[r._c(keep) for r in runs])
        res = (_Result * n)()
        arrs = []
        for i in range(n):
            r, a = _result_struct(runs[i].n_traj, lats[i].N, want_psi)
            res[i] = r
            arrs.append(a)
        _check(load().ihmc_run_batch(self.h, n, la, ra, res))
        return [_result_dict(res[i], arrs[i]) for i in range(n)]

    # ---- diagnostics
    def force(self, lat: Lattice, psi, precision=F32):
        keep = []
        psi = _f64(psi)
        F = np.zeros_like(psi)
        _check(load().ihmc_force(self.h, C.byref(lat._c(keep)), int(precision), _dp(psi), _dp(F)))
        return F

    def force_noalloc(self, lat: Lattice, psi_ptr, F_ptr, precision=F32, stream=None):
        """Allocation-free force on caller-owned device arrays (raw device
        pointers of N state-precision values each), enqueued on `stream` (raw
        hipStream_t; None or 0: the context stream); not synchronised."""
        keep = []
        _check(load().ihmc_force_noalloc(self.h, C.byref(lat._c(keep)), int(precision), C.c_void_p(psi_ptr),
                                         C.c_void_p(F_ptr), None if stream is None else C.c_void_p(stream)))

    def action(self, lat: Lattice, psi, precision=F32):
        keep = []
        psi = _f64(psi)
        out = np.zeros(5)
        _check(load().ihmc_action(self.h, C.byref(lat._c(keep)), int(precision), _dp(psi), _dp(out)))
        return dict(zip(("S", "m", "abs_m", "m2c", "beta_eps"), out.tolist()))

    def integrate(self, lat: Lattice, run: Run, psi, p):
        keep = []
        psi, p = _f64(psi).copy(), _f64(p).copy()
        _check(load().ihmc_integrate(self.h, C.byref(lat._c(keep)), C.byref(run._c(keep)), _dp(psi), _dp(p)))
        return psi, p

    def run_dense(self, model: Dense, runs, products=6, want_psi=True):
        keep = []
        n = len(runs)
        ra = (_Run * n)(*[r._c(keep) for r in runs])
        res = (_Result * n)()
        arrs = []
        for i in range(n):
            r, a = _result_struct(runs[i].n_traj, model.N, want_psi)
            res[i] = r
            arrs.append(a)
        _check(load().ihmc_run_dense(self.h, C.byref(model._c(keep)), n, ra, int(products), res))
        return [_result_dict(res[i], arrs[i]) for i in range(n)]

    def dense_force(self, model: Dense, psi, products=6):
        """Forces of the rows of psi (n x N) through the GEMM path."""
        keep = []
        psi = np.atleast_2d(_f64(psi))
        F = np.zeros_like(psi)
        _check(load().ihmc_dense_force(self.h, C.byref(model._c(keep)), psi.shape[0], _dp(psi), int(products),
                                       _dp(F)))
        return F

    def min_eig(self, K):
        """(theta, |r|, steps): lowest Ritz value of K by FP64 Lanczos and its residual norm."""
        K = np.ascontiguousarray(K, dtype=np.float64)
        th, rs, st = C.c_double(), C.c_double(), C.c_int32()
        _check(load().ihmc_min_eig(self.h, _dp(K), K.shape[0], C.byref(th), C.byref(rs), C.byref(st)))
        return th.value, rs.value, st.value

    def mh_run(self, lat: Lattice, n_sweeps, seed=0, chain_id=0, spins0=None):
        """Checkerboard single-spin Metropolis-Hastings on the GPU: dict(m, beta_eps
        (per sweep), spins (final, int8), acceptance, seconds (GPU time of the sweeps))."""
        keep = []
        N = lat.N
        m, be = np.zeros(max(1, n_sweeps)), np.zeros(max(1, n_sweeps))
        fin = np.zeros(N, dtype=np.int8)
        st = np.zeros(2)
        i8p = C.POINTER(C.c_int8)
        s0 = None if spins0 is None else np.ascontiguousarray(spins0, dtype=np.int8)
        _check(load().ihmc_mh_run(self.h, C.byref(lat._c(keep)), int(n_sweeps), int(seed), int(chain_id),
                                  None if s0 is None else s0.ctypes.data_as(i8p), _dp(m), _dp(be),
                                  fin.ctypes.data_as(i8p), _dp(st)))
        return dict(m=m[:n_sweeps], beta_eps=be[:n_sweeps], spins=fin, acceptance=float(st[0]),
                    seconds=float(st[1]))

    def dense_mh_run(self, model: "Dense", n_chains, n_sweeps, seed=0, chain_id=0, spins0=None):
        """Sequential single-spin Metropolis-Hastings with an explicit coupling
        matrix on the GPU, chains chain_id .. chain_id + n_chains - 1: dict(m,
        beta_eps (n_chains x n_sweeps), spins (n_chains x N, int8), acceptance
        (per chain), seconds (GPU time of the launch))."""
        keep = []
        N = model.N
        m = np.zeros((n_chains, max(1, n_sweeps)))
        be = np.zeros((n_chains, max(1, n_sweeps)))
        fin = np.zeros((n_chains, N), dtype=np.int8)
        acc = np.zeros(n_chains)
        sec = np.zeros(1)
        i8p = C.POINTER(C.c_int8)
        s0 = None
        if spins0 is not None:
            s0 = np.ascontiguousarray(np.broadcast_to(np.asarray(spins0, dtype=np.int8), (n_chains, N)))
        _check(load().ihmc_dense_mh_run(self.h, C.byref(model._c(keep)), int(n_chains), int(n_sweeps), int(seed),
                                        int(chain_id), None if s0 is None else s0.ctypes.data_as(i8p), _dp(m),
                                        _dp(be), fin.ctypes.data_as(i8p), _dp(acc), _dp(sec)))
        if n_sweeps == 0:
            m, be = m[:, :0], be[:, :0]
        return dict(m=np.ascontiguousarray(m), beta_eps=np.ascontiguousarray(be), spins=fin, acceptance=acc,
                    seconds=float(sec[0]))

    def copy_bandwidth(self, nbytes, reps=20):
        """Mean microseconds of one plain device copy of nbytes (2 * nbytes of traffic)."""
        us = C.c_double()
        _check(load().ihmc_copy_bandwidth(self.h, int(nbytes), int(reps), C.byref(us)))
        return us.value

    def philox_normals(self, seed, chain_id, traj, tag, n, precision=F64):
        """Normals of sites 0..n-1 as a pass of state `precision` draws them."""
        out = np.zeros(n)
        _check(load().ihmc_philox_normals(self.h, seed, chain_id, traj, tag, int(precision), n, _dp(out)))
        return out

    def hamiltonian(self, lat: Lattice, psi, p, precision=F64):
        """H(psi, p) = 1/2 p.p + S(psi) through the hot path's kernels (exact fixed-point sums)."""
        keep = []
        psi, p = _f64(psi), _f64(p)
        H = np.zeros(1)
        _check(load().ihmc_hamiltonian(self.h, C.byref(lat._c(keep)), int(precision), _dp(psi), _dp(p), _dp(H)))
        return float(H[0])

    def philox_words(self, ctr, key):
        ctr = np.ascontiguousarray(ctr, dtype=np.uint32).reshape(-1, 4)
        key = np.ascontiguousarray(key, dtype=np.uint32).reshape(-1, 2)
        n = ctr.shape[0]
        out = np.zeros((n, 4), dtype=np.uint32)
        u32 = C.POINTER(C.c_uint32)
        _check(load().ihmc_philox_words(self.h, n, ctr.ctypes.data_as(u32), key.ctypes.data_as(u32),
                                        out.ctypes.data_as(u32)))
        return out


def _checkpoint(fn, h, i):
    n = C.c_uint64(0)
    _check(fn(h, int(i), None, C.byref(n)))
    buf = C.create_string_buffer(n.value)
    _check(fn(h, int(i), buf, C.byref(n)))
    return buf.raw[:n.value]


class Chains:
    """Chains resident on the device; advance() enqueues trajectories asynchronously."""

    def __init__(self, ctx: Context, lats, runs):
        self.ctx = ctx
        keep = []
        n = len(lats)
        self.n = n
        self.lats, self.runs = list(lats), list(runs)
        la = (_Lattice * n)(*[l._c(keep) for l in lats])
        ra = (_Run * n)(*[r._c(keep) for r in runs])
        h = C.c_void_p()
        _check(load().ihmc_chains_create(ctx.h, n, la, ra, C.byref(h)))
        self.h = h

    def advance(self, n_traj):
        _check(load().ihmc_chains_advance(self.h, int(n_traj)))

    def result(self, i, want_psi=True):
        r, a = _result_struct(self.runs[i].n_traj, self.lats[i].N, want_psi)
        _check(load().ihmc_chains_result(self.h, int(i), C.byref(r)))
        return _result_dict(r, a)

    def checkpoint(self, i):
        """State of chain i after the queued trajectories, as bytes."""
        return _checkpoint(load().ihmc_chains_checkpoint, self.h, i)

    def restore(self, i, data):
        """Continue chain i from a checkpoint of a chain with the same parameters."""
        buf = C.create_string_buffer(bytes(data), len(data))
        _check(load().ihmc_chains_restore(self.h, int(i), buf, len(data)))

    def groups(self):
        n = C.c_int32()
        _check(load().ihmc_chains_groups(self.h, C.byref(n)))
        return n.value

    def group_info(self, group):
        """{'precision', 'ndim', 'cls', 'chains', 'sites', 'tiles'} of a launch group."""
        out = (C.c_int64 * 6)()
        _check(load().ihmc_chains_group_info(self.h, int(group), out))
        return dict(zip(("precision", "ndim", "cls", "chains", "sites", "tiles"), (int(v) for v in out)))

    def group_chains(self, group):
        """Indices of the chains of a launch group, in launch order."""
        n = self.group_info(group)["chains"]
        out = (C.c_int32 * max(1, n))()
        _check(load().ihmc_chains_group_chains(self.h, int(group), out))
        return [int(out[i]) for i in range(n)]

    def time_pass(self, group, mode=1, reps=50):
        """Mean duration (us) of one fused pass launch of a group, timed with HIP events
        (mode 0 first, 1 middle, 2 last, PAIR = two middle steps, 2D only)."""
        us, sites, nd, pr = C.c_double(), C.c_int64(), C.c_int32(), C.c_int32()
        _check(load().ihmc_chains_time_pass(self.h, int(group), int(mode), int(reps), C.byref(us),
                                            C.byref(sites), C.byref(nd), C.byref(pr)))
        return dict(us=us.value, sites=sites.value, ndim=nd.value, precision=pr.value)

    def close(self):
        if getattr(self, "h", None):
            load().ihmc_chains_destroy(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


class DenseChains:
    """Chains of one dense model, resident on the device; both K~ applications of
    every force evaluation run as GEMMs over all chains."""

    def __init__(self, ctx: Context, model: Dense, runs, products=6):
        self.ctx, self.model, self.runs = ctx, model, list(runs)
        keep = []
        n = len(runs)
        self.n = n
        ra = (_Run * n)(*[r._c(keep) for r in runs])
        h = C.c_void_p()
        _check(load().ihmc_dense_create(ctx.h, C.byref(model._c(keep)), n, ra, int(products), C.byref(h)))
        self.h = h

    def advance(self, n_traj):
        _check(load().ihmc_dense_advance(self.h, int(n_traj)))

    def result(self, i, want_psi=True):
        r, a = _result_struct(self.runs[i].n_traj, self.model.N, want_psi)
        _check(load().ihmc_dense_result(self.h, int(i), C.byref(r)))
        return _result_dict(r, a)

    def checkpoint(self, i):
        """State of chain i after the queued trajectories, as bytes."""
        return _checkpoint(load().ihmc_dense_checkpoint, self.h, i)

    def restore(self, i, data):
        """Continue chain i from a checkpoint of a chain of the same model and parameters."""
        buf = C.create_string_buffer(bytes(data), len(data))
        _check(load().ihmc_dense_restore(self.h, int(i), buf, len(data)))

    def info(self):
        out = np.zeros(5)
        _check(load().ihmc_dense_info(self.h, _dp(out)))
        return dict(C=out[0], theta=out[1], resid=out[2], lanczos_steps=int(out[3]), cg_iters=int(out[4]))

    def time(self, what=0, reps=20):
        """Mean microseconds of one launch: 0 BF16-limb GEMM, 1 FP64 GEMM, 2 whole force evaluation."""
        us = C.c_double()
        mnk = (C.c_int64 * 4)()
        _check(load().ihmc_dense_time(self.h, int(what), int(reps), C.byref(us), mnk))
        return dict(us=us.value, m=mnk[0], n=mnk[1], k=mnk[2], split_k=mnk[3])

    def close(self):
        if getattr(self, "h", None):
            load().ihmc_dense_destroy(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


class Server:
    """Continuous-batching server: submit() queues a lattice request, the
    library's scheduler thread admits it by HBM budget and advances all
    resident chains together; fetch() returns the results and timings."""

    STATS = ("rounds", "busy_s", "site_md_steps", "max_resident", "completed", "queued", "resident",
             "uptime_s", "bytes_held", "budget")

    def __init__(self, ctx: Context, budget_bytes=0, max_active=0):
        self.ctx = ctx
        h = C.c_void_p()
        _check(load().ihmc_server_create(ctx.h, int(budget_bytes), int(max_active), C.byref(h)))
        self.h = h
        self._meta = {}

    def submit(self, lat: Lattice, run: Run):
        keep = []
        t = C.c_uint64()
        _check(load().ihmc_submit(self.h, C.byref(lat._c(keep)), C.byref(run._c(keep)), C.byref(t)))
        self._meta[t.value] = (run.n_traj, lat.N)
        return t.value

    def poll(self, ticket):
        st = C.c_int32()
        _check(load().ihmc_poll(self.h, int(ticket), C.byref(st)))
        return st.value

    def wait(self, ticket, timeout=60.0):
        st = C.c_int32()
        _check(load().ihmc_wait(self.h, int(ticket), float(timeout), C.byref(st)))
        return st.value

    def info(self, ticket):
        """{'state', 'sites', 'n_traj', 'done'} of a request."""
        out = (C.c_int64 * 4)()
        _check(load().ihmc_request_info(self.h, int(ticket), out))
        return dict(zip(("state", "sites", "n_traj", "done"), (int(v) for v in out)))

    def checkpoint(self, ticket):
        """The request's checkpoint, as bytes (a running request: at the next
        round boundary; it keeps running)."""
        n = C.c_uint64(0)
        _check(load().ihmc_checkpoint(self.h, int(ticket), None, C.byref(n)))
        buf = C.create_string_buffer(n.value)
        _check(load().ihmc_checkpoint(self.h, int(ticket), buf, C.byref(n)))
        return buf.raw[:n.value]

    def restore(self, data):
        """Queue a request that continues from a checkpoint; returns its ticket."""
        buf = C.create_string_buffer(bytes(data), len(data))
        t = C.c_uint64()
        _check(load().ihmc_restore(self.h, buf, len(data), C.byref(t)))
        inf = self.info(t.value)
        self._meta[t.value] = (inf["n_traj"], inf["sites"])
        return t.value

    def fetch(self, ticket, want_psi=True):
        n_traj, N = self._meta[ticket]
        r, a = _result_struct(n_traj, N, want_psi)
        times = np.zeros(3)
        rc = load().ihmc_fetch(self.h, int(ticket), C.byref(r), _dp(times))
        if rc == IHMC_OK or rc == -5:
            self._meta.pop(ticket, None)
        _check(rc)
        out = _result_dict(r, a)
        out.update(t_submit=times[0], t_admit=times[1], t_done=times[2])
        return out

    def cancel(self, ticket):
        _check(load().ihmc_cancel(self.h, int(ticket)))

    def stats(self):
        out = np.zeros(10)
        _check(load().ihmc_server_stats(self.h, _dp(out)))
        return dict(zip(self.STATS, out.tolist()))

    def close(self):
        if getattr(self, "h", None):
            load().ihmc_server_destroy(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass
