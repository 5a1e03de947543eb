"""CPU oracle for the alchemical nonbonded path.

TEST INFRASTRUCTURE: only the tests, ``__graft_entry__.smoke()`` and the
benchmark's CPU-baseline leg use this package.  It never imports the GPU
library and the GPU library never imports it.

``alch_oracle.c`` holds the FP64 O(N^2) pair loop; ``opes.py`` and
``dihedral.py`` hold the FP64 reference for the lambda/OPES bias update and
the dihedral collective variables; ``ldyn.py`` and ``hrex.py`` the lambda
and d-AFED dynamics and the replica exchange; ``pme.py`` the particle-mesh
Ewald reciprocal space with the lambda-scaled solute-solvent cross term.
"""
from __future__ import annotations

import ctypes
import os
import subprocess
import threading

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "alch_oracle.c")
_LIB = os.path.join(_HERE, "liboracle.so")
_lock = threading.Lock()
_lib = None

BEUTLER, LBF = 0, 1
EWALD_REAL = 4
TERM_NAMES = ["E_solv_solv", "E_solu_solu", "E_ss_vdw", "E_ss_elec", "U_A", "U_B",
              "dUdl_vdw", "dUdl_elec", "E_total", "dUdl_total"]
NTERMS = len(TERM_NAMES)


def build(force: bool = False) -> str:
    """Compile the C oracle (gcc, FP64, no FMA contraction, OpenMP)."""
    if force or not os.path.exists(_LIB) or os.path.getmtime(_LIB) < os.path.getmtime(_SRC):
        tmp = _LIB + ".tmp%d" % os.getpid()
        subprocess.check_call(["gcc", "-O2", "-std=c11", "-D_DEFAULT_SOURCE", "-ffp-contract=off", "-fopenmp",
                               "-fPIC", "-shared", "-o", tmp, _SRC, "-lm"])
        os.replace(tmp, _LIB)
    return _LIB


def _load():
    global _lib
    with _lock:
        if _lib is None:
            build()
            lib = ctypes.CDLL(_LIB)
            P = ctypes.c_void_p
            d, i, i64 = ctypes.c_double, ctypes.c_int, ctypes.c_int64
            lib.oracle_eval.argtypes = [i, P, P, P, i, P, P, i, P, P, P, d, d, d, d, i, d, P, P, P, P, P, i]
            lib.oracle_eval.restype = i
            lib.oracle_pairs.argtypes = [i, P, i, P, P, d, P, i64, P]
            lib.oracle_pairs.restype = i
            lib.oracle_atom_energy.argtypes = [i, i, P, P, P, i, P, P, i, P, P, P, d, d, d, d, i, d]
            lib.oracle_atom_energy.restype = d
            lib.oracle_atoms_terms.argtypes = [i, P, i, P, P, P, i, P, P, i, P, P, P, d, d, d, d, i, d, P, P, P, P,
                                               i]
            lib.oracle_atoms_terms.restype = i
            lib.oracle_pair_probe.argtypes = [d, d, d, d, i, d, d, d, d, i, d, P]
            lib.oracle_pair_probe.restype = None
            lib.oracle_lbf_switches.argtypes = [d, P]
            lib.oracle_ucap.argtypes = [d, P]
            lib.oracle_switch.argtypes = [d, d, d, P]
            lib.oracle_dsf.argtypes = [d, d, d, P]
            lib.oracle_ewald_real.argtypes = [d, d, P]
            _lib = lib
    return _lib


def _ptr(a):
    return a.ctypes.data_as(ctypes.c_void_p) if a is not None else None


def _c(a, dtype):
    return np.ascontiguousarray(a, dtype=dtype)


class Params:
    """Pair-potential parameters of one evaluation."""

    def __init__(self, cutoff, switch_width=1.0, dsf_alpha=0.2, sc_alpha=0.5, schedule=BEUTLER, ewald=False):
        self.cutoff = float(cutoff)
        self.switch_width = float(switch_width)
        self.dsf_alpha = float(dsf_alpha)   # the Ewald splitting parameter when ewald is set
        self.sc_alpha = float(sc_alpha)
        self.schedule = int(schedule)
        self.ewald = bool(ewald)            # real-space Ewald erfc(a r)/r in place of D(r)

    @property
    def code(self):
        """The schedule argument of the C entry points (bit 2: Ewald real space)."""
        return self.schedule | (EWALD_REAL if self.ewald else 0)

    @classmethod
    def of(cls, workload, schedule=BEUTLER):
        return cls(workload.cutoff, workload.switch_width, workload.dsf_alpha, workload.sc_alpha, schedule)


def evaluate(positions, types, is_solute, exclusions, box, sigma, epsilon, charge, params: Params, lam,
             forces=True, param_grads=False, n_threads=0):
    """Evaluate one box.  Returns dict(terms, forces, pgrad, n_pairs)."""
    lib = _load()
    pos = _c(positions, np.float64).reshape(-1, 3)
    n = pos.shape[0]
    t = _c(types, np.int32)
    s = _c(is_solute, np.uint8)
    ex = _c(exclusions, np.int32).reshape(-1, 2)
    bx = _c(box, np.float64)
    sg, ep, ch = _c(sigma, np.float64), _c(epsilon, np.float64), _c(charge, np.float64)
    terms = np.zeros(NTERMS)
    f = np.zeros((n, 3)) if forces else None
    g = np.zeros((3, sg.shape[0])) if param_grads else None
    npairs = np.zeros(1, np.int64)
    absterms = np.zeros(NTERMS)
    rc = lib.oracle_eval(n, _ptr(pos), _ptr(t), _ptr(s), ex.shape[0], _ptr(ex), _ptr(bx), sg.shape[0], _ptr(sg),
                         _ptr(ep), _ptr(ch), params.cutoff, params.switch_width, params.dsf_alpha, params.sc_alpha,
                         params.code, float(lam), _ptr(terms), _ptr(f), _ptr(g), _ptr(npairs), _ptr(absterms),
                         int(n_threads))
    if rc != 0:
        raise ValueError("oracle_eval rejected its input (code %d)" % rc)
    out = dict(terms=terms, forces=f, n_pairs=int(npairs[0]), abs_terms=absterms)
    if param_grads:
        eps_t = ep
        with np.errstate(divide="ignore", invalid="ignore"):
            d_eps = np.where(eps_t > 0, g[1] / (2.0 * np.sqrt(np.where(eps_t > 0, eps_t, 1.0))), np.nan)
        out.update(d_sigma=g[0], d_sqrt_eps=g[1], d_eps=d_eps, d_charge=g[2])
    return out


def evaluate_system(system, ff, params: Params, lam, **kw):
    return evaluate(system.positions, system.types, system.is_solute, system.exclusions, system.box,
                    ff.sigma, ff.epsilon, ff.charge, params, lam, **kw)


def pair_set(positions, exclusions, box, r_list):
    """Sorted int32 [m, 2] list of i<j pairs within r_list (canonical test)."""
    lib = _load()
    pos = _c(positions, np.float64).reshape(-1, 3)
    ex = _c(exclusions, np.int32).reshape(-1, 2)
    bx = _c(box, np.float64)
    m = np.zeros(1, np.int64)
    rc = lib.oracle_pairs(pos.shape[0], _ptr(pos), ex.shape[0], _ptr(ex), _ptr(bx), float(r_list), None, 0, _ptr(m))
    if rc != 0:
        raise ValueError("oracle_pairs rejected its input (code %d)" % rc)
    out = np.zeros((int(m[0]), 2), np.int32)
    rc = lib.oracle_pairs(pos.shape[0], _ptr(pos), ex.shape[0], _ptr(ex), _ptr(bx), float(r_list), _ptr(out),
                          int(m[0]), _ptr(m))
    if rc != 0:
        raise ValueError("oracle_pairs failed (code %d)" % rc)
    return out


def atom_energy(a, system, ff, params: Params, lam, positions=None):
    lib = _load()
    pos = _c(system.positions if positions is None else positions, np.float64).reshape(-1, 3)
    t = _c(system.types, np.int32)
    s = _c(system.is_solute, np.uint8)
    ex = _c(system.exclusions, np.int32).reshape(-1, 2)
    bx = _c(system.box, np.float64)
    sg, ep, ch = _c(ff.sigma, np.float64), _c(ff.epsilon, np.float64), _c(ff.charge, np.float64)
    return lib.oracle_atom_energy(int(a), pos.shape[0], _ptr(pos), _ptr(t), _ptr(s), ex.shape[0], _ptr(ex),
                                  _ptr(bx), sg.shape[0], _ptr(sg), _ptr(ep), _ptr(ch), params.cutoff,
                                  params.switch_width, params.dsf_alpha, params.sc_alpha, params.code,
                                  float(lam))


def atoms_terms(sel, system, ff, params: Params, lam, positions=None, n_threads=0):
    """Per-atom sums for the atoms in sel: dict(forces [S,3] = -dU/dx_a, energy [S]
    (pair energies involving a), dudl [S] (its solute-solvent pairs), n_pairs [S])."""
    lib = _load()
    sl = _c(sel, np.int32)
    pos = _c(system.positions if positions is None else positions, np.float64).reshape(-1, 3)
    t = _c(system.types, np.int32)
    s = _c(system.is_solute, np.uint8)
    ex = _c(system.exclusions, np.int32).reshape(-1, 2)
    bx = _c(system.box, np.float64)
    sg, ep, ch = _c(ff.sigma, np.float64), _c(ff.epsilon, np.float64), _c(ff.charge, np.float64)
    S = sl.shape[0]
    f, e, dl, npair = np.zeros((S, 3)), np.zeros(S), np.zeros(S), np.zeros(S, np.int64)
    rc = lib.oracle_atoms_terms(S, _ptr(sl), pos.shape[0], _ptr(pos), _ptr(t), _ptr(s), ex.shape[0], _ptr(ex),
                                _ptr(bx), sg.shape[0], _ptr(sg), _ptr(ep), _ptr(ch), params.cutoff,
                                params.switch_width, params.dsf_alpha, params.sc_alpha, params.code, float(lam),
                                _ptr(f), _ptr(e), _ptr(dl), _ptr(npair), int(n_threads))
    if rc != 0:
        raise ValueError("oracle_atoms_terms rejected its input (code %d)" % rc)
    return dict(forces=f, energy=e, dudl=dl, n_pairs=npair)


def pair_probe(r, sig, eps, qq, alchemical, params: Params, lam):
    """One pair: (u, -du/dr, du/dlambda, du/dsig, du/deps, du/dqq)."""
    lib = _load()
    out = np.zeros(6)
    lib.oracle_pair_probe(float(r), float(sig), float(eps), float(qq), int(bool(alchemical)), params.cutoff,
                          params.switch_width, params.dsf_alpha, params.sc_alpha, params.code, float(lam),
                          _ptr(out))
    return out


def lbf_switches(lam):
    out = np.zeros(4)
    _load().oracle_lbf_switches(float(lam), _ptr(out))
    return out


def ucap(x):
    out = np.zeros(2)
    _load().oracle_ucap(float(x), _ptr(out))
    return out


def switch(r, rc, width):
    out = np.zeros(2)
    _load().oracle_switch(float(r), float(rc), float(width), _ptr(out))
    return out


def dsf(r, rc, alpha):
    out = np.zeros(2)
    _load().oracle_dsf(float(r), float(rc), float(alpha), _ptr(out))
    return out


def ewald_real(r, alpha):
    """erfc(alpha r)/r and its r derivative (the real-space Ewald kernel)."""
    out = np.zeros(2)
    _load().oracle_ewald_real(float(r), float(alpha), _ptr(out))
    return out
