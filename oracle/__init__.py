"""FP64 CPU oracle for HMC on the Hubbard-Stratonovich-transformed Ising model.

TEST INFRASTRUCTURE.  Only ``tests/``, ``__graft_entry__.smoke()`` and the
``cpu_baseline`` leg of ``bench.py`` may import this package.  The product
path (``paper_1912_03278_amd``) never imports it, and it never imports the
product path: the two share no code.

``oracle/ihmc_oracle.c`` holds the arithmetic (plain loops, FP64, Neumaier
sums); this module is a ctypes wrapper around it.  ``oracle.exact`` holds the
exact references (brute force, transfer matrices, closed forms) and
``oracle.stats`` the Gamma-method error analysis.

Paper: Ostmeyer et al., "The Ising Model with Hybrid Monte Carlo",
arXiv:1912.03278 -- Sec. 2 (transformation), Sec. 3 (HMC), Sec. 4
(estimators), App. A (infinite-range model).
"""
from __future__ import annotations

import ctypes as C
import os
import subprocess
from dataclasses import dataclass, field

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "ihmc_oracle.c")
_LIB = os.path.join(_HERE, "liboracle_ihmc.so")

TAG_INIT, TAG_MOM, TAG_ACC, TAG_FLIP, TAG_MH, TAG_MH_INIT = 1, 2, 3, 4, 5, 6
LEAPFROG, OMELYAN = 0, 1


def build() -> str:
    """Compile the oracle with gcc (no fast-math, no FP contraction)."""
    cmd = ["gcc", "-O2", "-std=c99", "-fPIC", "-shared", "-ffp-contract=off",
           "-fno-fast-math", _SRC, "-o", _LIB + ".tmp", "-lm"]
    subprocess.run(cmd, check=True)
    os.replace(_LIB + ".tmp", _LIB)
    return _LIB


class _Lattice(C.Structure):
    _fields_ = [("ndim", C.c_int32), ("L", C.c_int32 * 3), ("J", C.c_double),
                ("beta", C.c_double), ("C", C.c_double), ("h", C.POINTER(C.c_double)),
                ("h_len", C.c_int64)]


class _Dense(C.Structure):
    _fields_ = [("N", C.c_int64), ("K", C.POINTER(C.c_double)), ("J", C.c_double),
                ("beta", C.c_double), ("C", C.c_double), ("h", C.POINTER(C.c_double)),
                ("h_len", C.c_int64)]


class _Run(C.Structure):
    _fields_ = [("n_md", C.c_int32), ("traj_len", C.c_double), ("n_traj", C.c_int32),
                ("flip_every", C.c_int32), ("integrator", C.c_int32), ("form", C.c_int32),
                ("seed", C.c_uint64), ("chain_id", C.c_uint64),
                ("psi0", C.POINTER(C.c_double)), ("replay_accept", C.POINTER(C.c_uint8))]


class _Result(C.Structure):
    _fields_ = [("dH", C.POINTER(C.c_double)), ("m", C.POINTER(C.c_double)),
                ("abs_m", C.POINTER(C.c_double)), ("m2c", C.POINTER(C.c_double)),
                ("beta_eps", C.POINTER(C.c_double)), ("H_old", C.POINTER(C.c_double)),
                ("H_new", C.POINTER(C.c_double)), ("accepted", C.POINTER(C.c_uint8)),
                ("flipped", C.POINTER(C.c_uint8)), ("psi_final", C.POINTER(C.c_double)),
                ("acceptance", C.c_double), ("mean_exp_minus_dH", C.c_double),
                ("n_nonfinite", C.c_int64)]


_lib = None


def lib():
    global _lib
    if _lib is None:
        if not os.path.exists(_LIB) or os.path.getmtime(_LIB) < os.path.getmtime(_SRC):
            build()
        L = C.CDLL(_LIB)
        dp = C.POINTER(C.c_double)
        lp, dnp = C.POINTER(_Lattice), C.POINTER(_Dense)
        L.orc_philox4x32_10.argtypes = [C.POINTER(C.c_uint32), C.POINTER(C.c_uint32), C.POINTER(C.c_uint32)]
        L.orc_uniform.argtypes = [C.c_uint64, C.c_uint64, C.c_uint32, C.c_uint32]
        L.orc_uniform.restype = C.c_double
        L.orc_normals.argtypes = [C.c_uint64, C.c_uint64, C.c_uint32, C.c_uint32, C.c_int64, dp]
        L.orc_lattice_apply.argtypes = [lp, dp, dp]
        L.orc_dense_apply.argtypes = [dnp, dp, dp]
        L.orc_force.argtypes = [lp, dnp, dp, dp]
        L.orc_action.argtypes = [lp, dnp, dp, dp]
        L.orc_hamiltonian.argtypes = [lp, dnp, dp, dp, dp]
        L.orc_md.argtypes = [lp, dnp, C.c_int32, C.c_double, C.c_int32, dp, dp]
        L.orc_constants.argtypes = [lp, dnp, dp]
        L.orc_shifted_force.argtypes = [lp, dnp, dp, dp]
        L.orc_shifted_action.argtypes = [lp, dnp, dp, dp]
        L.orc_shifted_md.argtypes = [lp, dnp, C.c_int32, C.c_double, C.c_int32, dp, dp]
        L.orc_run_lattice.argtypes = [lp, C.POINTER(_Run), C.POINTER(_Result)]
        L.orc_run_dense.argtypes = [dnp, C.POINTER(_Run), C.POINTER(_Result)]
        L.orc_phi_force.argtypes = [lp, dnp, dp, dp]
        L.orc_phi_action.argtypes = [lp, dnp, dp, dp]
        L.orc_phi_start.argtypes = [lp, dnp, C.POINTER(_Run), dp]
        L.orc_phi_md.argtypes = [lp, dnp, C.c_int32, C.c_double, dp, dp]
        L.orc_run_phi.argtypes = [lp, dnp, C.POINTER(_Run), C.POINTER(_Result)]
        i8p = C.POINTER(C.c_int8)
        L.orc_mh_run.argtypes = [lp, C.c_int32, C.c_uint64, C.c_uint64, i8p, dp, dp, i8p, dp]
        L.orc_dense_mh_run.argtypes = [dnp, C.c_int32, C.c_uint64, C.c_uint64, i8p, dp, dp, i8p, dp]
        _lib = L
    return _lib


def _dp(a):
    return a.ctypes.data_as(C.POINTER(C.c_double)) if a is not None else None


def _f64(a):
    return None if a is None else np.ascontiguousarray(a, dtype=np.float64)


@dataclass
class Lattice:
    """Periodic hypercubic nearest-neighbour Ising model (Sec. 2)."""
    L: tuple
    beta: float
    C: float
    J: float = 1.0
    h: object = None  # None, scalar, or array of N site fields

    @property
    def ndim(self):
        return len(self.L)

    @property
    def N(self):
        return int(np.prod(self.L))

    def _c(self):
        h = None if self.h is None else _f64(np.atleast_1d(self.h))
        s = _Lattice()
        s.ndim = self.ndim
        for i in range(3):
            s.L[i] = int(self.L[i]) if i < self.ndim else 1
        s.J, s.beta, s.C = float(self.J), float(self.beta), float(self.C)
        s.h = _dp(h)
        s.h_len = 0 if h is None else h.size
        return s, h  # keep h alive


@dataclass
class Dense:
    """Explicit symmetric coupling matrix in place of J*K (Sec. 2, App. A)."""
    K: np.ndarray
    beta: float
    C: float
    J: float = 1.0
    h: object = None

    @property
    def N(self):
        return int(self.K.shape[0])

    def _c(self):
        K = _f64(self.K)
        h = None if self.h is None else _f64(np.atleast_1d(self.h))
        s = _Dense()
        s.N = K.shape[0]
        s.K = _dp(K)
        s.J, s.beta, s.C = float(self.J), float(self.beta), float(self.C)
        s.h = _dp(h)
        s.h_len = 0 if h is None else h.size
        return s, (K, h)


def _model(model):
    s, keep = model._c()
    if isinstance(model, Lattice):
        return C.byref(s), None, (s, keep)
    return None, C.byref(s), (s, keep)


def philox4x32_10(ctr, key):
    c = (C.c_uint32 * 4)(*[int(v) & 0xFFFFFFFF for v in ctr])
    k = (C.c_uint32 * 2)(*[int(v) & 0xFFFFFFFF for v in key])
    o = (C.c_uint32 * 4)()
    lib().orc_philox4x32_10(c, k, o)
    return np.array(list(o), dtype=np.uint32)


def normals(seed, chain, traj, tag, n):
    out = np.empty(n, dtype=np.float64)
    lib().orc_normals(seed, chain, traj, tag, n, _dp(out))
    return out


def uniform(seed, chain, traj, tag):
    return lib().orc_uniform(seed, chain, traj, tag)


FORMS = {"psi": 0, "shifted": 2}


def _shifted(form):
    if form not in FORMS:
        raise ValueError("form must be 'psi' or 'shifted'")
    return form == "shifted"


def apply_Kt(model, psi):
    psi = _f64(psi)
    u = np.empty_like(psi)
    a, d, keep = _model(model)
    rc = lib().orc_lattice_apply(a, _dp(psi), _dp(u)) if a is not None else \
        lib().orc_dense_apply(d, _dp(psi), _dp(u))
    if rc:
        raise ValueError("invalid model")
    return u


def force(model, psi, form="psi"):
    """F = -dS/dpsi; form "shifted": the action with h' inside the log cosh."""
    psi = _f64(psi)
    F = np.empty_like(psi)
    a, d, keep = _model(model)
    fn = lib().orc_shifted_force if _shifted(form) else lib().orc_force
    if fn(a, d, _dp(psi), _dp(F)):
        raise ValueError("invalid model")
    return F


ACTION_KEYS = ("S", "m", "abs_m", "m2c", "beta_eps", "sum_psi", "sum_psih", "sum_ut")


def action(model, psi, form="psi"):
    """S(psi) and the per-configuration estimators (dict).  For the shifted
    form sum_ut holds sum y tanh(y), y = sqrt(J') Kt psi + h'."""
    psi = _f64(psi)
    out = np.empty(8)
    a, d, keep = _model(model)
    fn = lib().orc_shifted_action if _shifted(form) else lib().orc_action
    if fn(a, d, _dp(psi), _dp(out)):
        raise ValueError("invalid model")
    return dict(zip(ACTION_KEYS, out.tolist()))


def hamiltonian(model, psi, p):
    psi, p = _f64(psi), _f64(p)
    H = C.c_double()
    a, d, keep = _model(model)
    if lib().orc_hamiltonian(a, d, _dp(psi), _dp(p), C.byref(H)):
        raise ValueError("invalid model")
    return H.value


def md(model, psi, p, n_md, traj_len=1.0, integrator=LEAPFROG, form="psi"):
    """Integrate one trajectory; returns new (psi, p) copies."""
    psi, p = _f64(psi).copy(), _f64(p).copy()
    a, d, keep = _model(model)
    fn = lib().orc_shifted_md if _shifted(form) else lib().orc_md
    if fn(a, d, int(n_md), float(traj_len), int(integrator), _dp(psi), _dp(p)):
        raise ValueError("invalid model")
    return psi, p


def constants(model):
    """(1^T Kt^-1 h', h'^T Kt^-1 h', 1^T Kt^-1 1)."""
    out = np.empty(3)
    a, d, keep = _model(model)
    if lib().orc_constants(a, d, _dp(out)):
        raise ValueError("invalid model")
    return tuple(out.tolist())


# ---- the inverse (phi) formulation, eq. cosh_in_exponent (Sec. 2)

PHI_ACTION_KEYS = ("S", "m", "abs_m", "m2c", "beta_eps")


def phi_force(model, phi):
    """-dS/dphi = -Kt^-1 phi / J' + tanh(h' + phi) (one CG solve)."""
    phi = _f64(phi)
    F = np.empty_like(phi)
    a, d, keep = _model(model)
    if lib().orc_phi_force(a, d, _dp(phi), _dp(F)):
        raise ValueError("invalid model")
    return F


def phi_action(model, phi):
    """S(phi) and the spin estimators given phi (dict)."""
    phi = _f64(phi)
    out = np.empty(5)
    a, d, keep = _model(model)
    if lib().orc_phi_action(a, d, _dp(phi), _dp(out)):
        raise ValueError("invalid model")
    return dict(zip(PHI_ACTION_KEYS, out.tolist()))


def phi_start(model, seed=0, chain_id=0, psi0=None):
    """The phi chain's starting field sqrt(J') Kt psi0 - h' (psi0 from TAG_INIT unless given)."""
    r = _Run()
    r.seed, r.chain_id = int(seed), int(chain_id)
    p0 = _f64(psi0)
    r.psi0 = _dp(p0)
    out = np.empty(model.N)
    a, d, keep = _model(model)
    if lib().orc_phi_start(a, d, C.byref(r), _dp(out)):
        raise ValueError("invalid model")
    return out


def phi_md(model, phi, p, n_md, traj_len=1.0):
    """One leap-frog trajectory in phi; returns new (phi, p) copies."""
    phi, p = _f64(phi).copy(), _f64(p).copy()
    a, d, keep = _model(model)
    if lib().orc_phi_md(a, d, int(n_md), float(traj_len), _dp(phi), _dp(p)):
        raise ValueError("invalid model")
    return phi, p


def phi_hamiltonian(model, phi, p):
    return 0.5 * float(np.dot(p, p)) + phi_action(model, phi)["S"]


def mh_run(lat, n_sweeps, seed=0, chain_id=0, spins0=None):
    """Checkerboard single-spin Metropolis-Hastings (the comparison method of
    Sec. 4) on an even-extent periodic lattice with h = 0 or uniform: returns
    dict(m, beta_eps (per sweep), spins (final, int8), acceptance)."""
    s, keep = lat._c()
    N = lat.N
    m, be = np.zeros(n_sweeps), np.zeros(n_sweeps)
    fin = np.zeros(N, dtype=np.int8)
    s0 = None if spins0 is None else np.ascontiguousarray(spins0, dtype=np.int8)
    acc = C.c_double()
    i8p = C.POINTER(C.c_int8)
    rc = lib().orc_mh_run(C.byref(s), int(n_sweeps), int(seed), int(chain_id),
                          None if s0 is None else s0.ctypes.data_as(i8p), _dp(m), _dp(be),
                          fin.ctypes.data_as(i8p), C.byref(acc))
    if rc:
        raise ValueError("invalid lattice for checkerboard Metropolis-Hastings")
    return dict(m=m, beta_eps=be, spins=fin, acceptance=acc.value)


def dense_mh_run(model, n_sweeps, seed=0, chain_id=0, spins0=None):
    """Sequential single-spin Metropolis-Hastings with an explicit coupling
    matrix (sites in order 0 .. N-1, the local field summed afresh for every
    proposal): returns dict(m, beta_eps (per sweep), spins (final, int8),
    acceptance)."""
    s, keep = model._c()
    N = model.N
    m, be = np.zeros(n_sweeps), np.zeros(n_sweeps)
    fin = np.zeros(N, dtype=np.int8)
    s0 = None if spins0 is None else np.ascontiguousarray(spins0, dtype=np.int8)
    acc = C.c_double()
    i8p = C.POINTER(C.c_int8)
    rc = lib().orc_dense_mh_run(C.byref(s), int(n_sweeps), int(seed), int(chain_id),
                                None if s0 is None else s0.ctypes.data_as(i8p), _dp(m), _dp(be),
                                fin.ctypes.data_as(i8p), C.byref(acc))
    if rc:
        raise ValueError("invalid model for dense Metropolis-Hastings")
    return dict(m=m, beta_eps=be, spins=fin, acceptance=acc.value)


@dataclass
class RunResult:
    dH: np.ndarray
    accepted: np.ndarray
    flipped: np.ndarray
    m: np.ndarray
    abs_m: np.ndarray
    m2c: np.ndarray
    beta_eps: np.ndarray
    H_old: np.ndarray
    H_new: np.ndarray
    psi_final: np.ndarray
    acceptance: float
    mean_exp_minus_dH: float
    n_nonfinite: int


def run(model, n_traj, n_md, traj_len=1.0, seed=0, chain_id=0, psi0=None,
        replay_accept=None, flip_every=0, integrator=LEAPFROG, form="psi") -> RunResult:
    """A full HMC chain (Sec. 3), recording the estimators after each trajectory.
    form "psi": the substituted field (eq. phi_psi_substitution), psi0 the
    starting psi; form "phi": the inverse formulation (eq. cosh_in_exponent,
    leap-frog only, no flips), psi0 then the starting phi (None: the TAG_INIT
    psi0 mapped by phi = sqrt(J') Kt psi0 - h'); psi_final holds the final phi;
    form "shifted": the substitution phi = sqrt(J') Kt psi (h' inside the log
    cosh; flips only at h = 0)."""
    N = model.N
    out = {k: np.zeros(n_traj) for k in ("dH", "m", "abs_m", "m2c", "beta_eps", "H_old", "H_new")}
    acc = np.zeros(n_traj, dtype=np.uint8)
    flp = np.zeros(n_traj, dtype=np.uint8)
    psi_final = np.zeros(N)
    r = _Run()
    r.n_md, r.traj_len, r.n_traj = int(n_md), float(traj_len), int(n_traj)
    r.flip_every, r.integrator = int(flip_every), int(integrator)
    r.seed, r.chain_id = int(seed), int(chain_id)
    if form != "phi":
        r.form = FORMS[form] if form in FORMS else -1
    p0 = _f64(psi0)
    r.psi0 = _dp(p0)
    ra = None if replay_accept is None else np.ascontiguousarray(replay_accept, dtype=np.uint8)
    r.replay_accept = None if ra is None else ra.ctypes.data_as(C.POINTER(C.c_uint8))
    res = _Result()
    for k, v in out.items():
        setattr(res, k, _dp(v))
    res.accepted = acc.ctypes.data_as(C.POINTER(C.c_uint8))
    res.flipped = flp.ctypes.data_as(C.POINTER(C.c_uint8))
    res.psi_final = _dp(psi_final)
    a, d, keep = _model(model)
    if form == "phi":
        rc = lib().orc_run_phi(a, d, C.byref(r), C.byref(res))
    else:
        rc = lib().orc_run_lattice(a, C.byref(r), C.byref(res)) if a is not None else \
            lib().orc_run_dense(d, C.byref(r), C.byref(res))
    if rc:
        raise ValueError("invalid model or run parameters")
    return RunResult(accepted=acc, flipped=flp, psi_final=psi_final, acceptance=res.acceptance,
                     mean_exp_minus_dH=res.mean_exp_minus_dH, n_nonfinite=res.n_nonfinite, **out)
