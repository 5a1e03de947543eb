"""Python binding of libalchnb (ctypes; argument marshalling only).

Every computation runs in the HIP library; PyTorch supplies device memory and
the stream.  Importing this module loads ``libalchnb.so`` built in-tree by
``paper_2608_12691_amd.build`` and raises if it is missing: there is no
fallback path.
"""
from __future__ import annotations

import ctypes
import os
from typing import Optional, Sequence

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.environ.get("ALCHNB_LIB") or os.path.join(_HERE, "libalchnb.so")

BEUTLER_DSF, LBF_DSF = 0, 1
FP32_FIXED, FP64 = 0, 1
ELEC_DSF, ELEC_PME = 0, 1
AUTO_REBUILD, FORCE_REBUILD = 1, 2
FLAG_FIXED_OVERFLOW, FLAG_SKIN_EXCEEDED, FLAG_NONFINITE, FLAG_LAMBDA_RANGE, FLAG_CAPACITY = 1, 2, 4, 8, 16
FLAG_BARRIER_TIMEOUT, FLAG_BAD_INDEX, FLAG_LD_CAPACITY = 32, 64, 128
LIST_AUTO, LIST_PHASES, LIST_FUSED_ACTIVE = 0, 1, 2
NTERMS = 10
TERM_NAMES = ["E_solv_solv", "E_solu_solu", "E_ss_vdw", "E_ss_elec", "U_A", "U_B", "dUdl_vdw", "dUdl_elec",
              "E_total", "dUdl_total"]
OPES_GRID = 101
OPES_HEADER = 16

STATUS = {0: "ok", 1: "invalid argument", 2: "box too small", 3: "unsupported", 4: "capacity", 5: "hip error",
          6: "not bound", 7: "no device", 8: "workspace exceeds the static scratch"}

EXPORTED = ["alch_nb_create", "alch_nb_pme_grid", "alch_nb_workspace_size", "alch_nb_bind", "alch_nb_bind_static", "alch_nb_build_list", "alch_nb_compute",
            "alch_nb_backward", "alch_nb_dihedrals", "alch_nb_opes_update", "alch_nb_opes_layout", "alch_nb_opes_init", "alch_nb_opes_state_size",
            "alch_nb_ld_state_size", "alch_nb_ld_layout", "alch_nb_ld_init", "alch_nb_ld_step", "alch_nb_ld_step_dafed",
            "alch_nb_ld_free_energy", "alch_nb_hrex_init", "alch_nb_hrex_exchange", "alch_nb_capture_begin",
            "alch_nb_capture_end", "alch_nb_export_pairs", "alch_nb_capture_step", "alch_nb_launch_step", "alch_nb_autotune",
            "alch_nb_set_variant", "alch_nb_num_variants", "alch_nb_set_list_mode", "alch_nb_get_list_mode",
            "alch_nb_set_timing", "alch_nb_get_flags",
            "alch_nb_get_stats", "alch_nb_destroy", "alch_nb_strerror", "alch_nb_last_hip_error",
            "alch_nb_flops_per_pair"]


class AlchNBError(RuntimeError):
    def __init__(self, where, status, hip=0):
        self.status = status
        super().__init__("%s failed: %s (status %d%s)" % (where, STATUS.get(status, "?"), status,
                                                         ", hip error %d" % hip if hip else ""))


class System_t(ctypes.Structure):
    _fields_ = [("n_atoms", ctypes.c_int32), ("type", ctypes.c_void_p), ("is_solute", ctypes.c_void_p),
                ("n_excl", ctypes.c_int32), ("excl", ctypes.c_void_p), ("box", ctypes.c_double * 3)]


class Params_t(ctypes.Structure):
    _fields_ = [("n_types", ctypes.c_int32), ("sigma", ctypes.c_void_p), ("epsilon", ctypes.c_void_p),
                ("charge", ctypes.c_void_p), ("cutoff", ctypes.c_double), ("skin", ctypes.c_double),
                ("switch_width", ctypes.c_double), ("dsf_alpha", ctypes.c_double), ("sc_alpha", ctypes.c_double),
                ("schedule", ctypes.c_int32), ("precision", ctypes.c_int32), ("variant", ctypes.c_int32),
                ("list_capacity_factor", ctypes.c_double), ("electrostatics", ctypes.c_int32),
                ("pme_order", ctypes.c_int32), ("pme_spacing", ctypes.c_double)]


class Out_t(ctypes.Structure):
    _fields_ = [("terms", ctypes.c_void_p), ("forces", ctypes.c_void_p), ("dudl", ctypes.c_void_p),
                ("n_pairs", ctypes.c_void_p)]


class Grad_t(ctypes.Structure):
    _fields_ = [("d_pos", ctypes.c_void_p), ("d_lambda", ctypes.c_void_p), ("d_sigma", ctypes.c_void_p),
                ("d_sqrt_epsilon", ctypes.c_void_p), ("d_charge", ctypes.c_void_p), ("d_epsilon", ctypes.c_void_p)]


class LdParams_t(ctypes.Structure):
    _fields_ = [("capacity", ctypes.c_int32), ("stride", ctypes.c_int32), ("ti_bins", ctypes.c_int32),
                ("n_cv", ctypes.c_int32), ("kT", ctypes.c_double), ("mass", ctypes.c_double),
                ("friction", ctypes.c_double), ("dt", ctypes.c_double), ("sigma", ctypes.c_double),
                ("barrier_std", ctypes.c_double), ("barrier_expl", ctypes.c_double), ("compress", ctypes.c_double),
                ("kT_s", ctypes.c_double), ("friction_s", ctypes.c_double)]


LD_LAYOUT = ["rep0", "rep_stride", "theta", "p", "lambda", "last_lambda", "u_opes", "du_opes", "f_theta", "n",
             "n_std", "n_expl", "kern_std", "kern_expl", "ti", "cv_s", "cv_p", "cv_force"]


class Stats_t(ctypes.Structure):
    _fields_ = [("n_atoms", ctypes.c_int64), ("n_systems", ctypes.c_int64), ("n_superclusters", ctypes.c_int64),
                ("n_entries", ctypes.c_int64), ("n_units", ctypes.c_int64), ("entry_capacity", ctypes.c_int64),
                ("unit_capacity", ctypes.c_int64), ("n_rebuilds", ctypes.c_int64), ("n_tiles", ctypes.c_int64),
                ("variant", ctypes.c_int32),
                ("entries_per_unit", ctypes.c_int32), ("blocks", ctypes.c_int32), ("tile_ms_total", ctypes.c_double),
                ("tile_launches_timed", ctypes.c_int64)]


_lib = None


def load():
    """Load libalchnb.so (raises if it was not built)."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise ImportError("libalchnb.so is not built; run `python -m paper_2608_12691_amd.build`")
        lib = ctypes.CDLL(LIB_PATH)
        P, I32, I64, D, U32 = ctypes.c_void_p, ctypes.c_int32, ctypes.c_int64, ctypes.c_double, ctypes.c_uint32
        sig = {
            "alch_nb_create": ([P, P, I32, P], I32),
            "alch_nb_workspace_size": ([P, P], I32),
            "alch_nb_pme_grid": ([P, I32, P], I32),
            "alch_nb_bind": ([P, P, ctypes.c_size_t, P], I32),
            "alch_nb_bind_static": ([P, P], I32),
            "alch_nb_build_list": ([P, P], I32),
            "alch_nb_compute": ([P, P, P, U32, P], I32),
            "alch_nb_backward": ([P, P, P, P, P], I32),
            "alch_nb_dihedrals": ([P, P, I32, P, P, P, P, P, P, P, P, P], I32),
            "alch_nb_opes_update": ([P, P, P, P, I32], I32),
            "alch_nb_opes_layout": ([P, I32], I32),
            "alch_nb_opes_init": ([P, P, I32, D, D, D, D, D], I32),
            "alch_nb_opes_state_size": ([I32], I64),
            "alch_nb_ld_state_size": ([P, I32], I64),
            "alch_nb_ld_layout": ([P, I32, P, I32], I32),
            "alch_nb_ld_init": ([P, P, P, P, P, P, P], I32),
            "alch_nb_ld_step": ([P, P, P, P, P, I32, P], I32),
            "alch_nb_ld_step_dafed": ([P, P, P, P, P, P, P, P, P, I32, P], I32),
            "alch_nb_ld_free_energy": ([P, P, P], I32),
            "alch_nb_hrex_init": ([P, P, P], I32),
            "alch_nb_hrex_exchange": ([P, P, P, P, P, P, I32, D, P], I32),
            "alch_nb_capture_begin": ([P], I32),
            "alch_nb_capture_end": ([P], I32),
            "alch_nb_export_pairs": ([P, P, I64, P], I32),
            "alch_nb_capture_step": ([P, P, P, P], I32),
            "alch_nb_launch_step": ([P], I32),
            "alch_nb_autotune": ([P, P, P, I32], I32),
            "alch_nb_set_variant": ([P, I32], I32),
            "alch_nb_num_variants": ([], I32),
            "alch_nb_set_list_mode": ([P, I32], I32),
            "alch_nb_get_list_mode": ([P], I32),
            "alch_nb_set_timing": ([P, I32], I32),
            "alch_nb_get_flags": ([P, P], I32),
            "alch_nb_get_stats": ([P, P], I32),
            "alch_nb_destroy": ([P], None),
            "alch_nb_strerror": ([I32], ctypes.c_char_p),
            "alch_nb_last_hip_error": ([P], I32),
            "alch_nb_flops_per_pair": ([I32], D),
        }
        for name, (args, res) in sig.items():
            fn = getattr(lib, name)
            fn.argtypes = args
            fn.restype = res
        _lib = lib
    return _lib


def _addr(t) -> Optional[int]:
    if t is None:
        return None
    return t.data_ptr()


class Context:
    """One library context: K boxes sharing one parameter set.

    ``systems`` are objects with positions/types/is_solute/exclusions/box
    (see ``paper_2608_12691_amd.systems``); ``ff`` has sigma/epsilon/charge.
    """

    def __init__(self, ff, systems: Sequence, cutoff, skin, switch_width=1.0, dsf_alpha=0.2, sc_alpha=0.5,
                 schedule=BEUTLER_DSF, precision=FP32_FIXED, variant=-1, capacity_factor=1.0, device=None,
                 auto_capacity=True, static_scratch=False, electrostatics=ELEC_DSF, pme_order=5, pme_spacing=1.0):
        import torch
        self.torch = torch
        self.lib = load()
        self.device = torch.device(device or "cuda:0")
        self.schedule, self.precision = int(schedule), int(precision)
        self.K = len(systems)
        self.n_atoms = [int(s.positions.shape[0]) for s in systems]
        self.N = sum(self.n_atoms)
        self.n_types = len(ff.sigma)
        self._keep = []
        self._sys = (System_t * self.K)()
        for k, s in enumerate(systems):
            t = np.ascontiguousarray(s.types, np.int32)
            sol = np.ascontiguousarray(s.is_solute, np.uint8)
            ex = np.ascontiguousarray(s.exclusions, np.int32).reshape(-1, 2)
            self._keep += [t, sol, ex]
            self._sys[k].n_atoms = len(t)
            self._sys[k].type = t.ctypes.data
            self._sys[k].is_solute = sol.ctypes.data
            self._sys[k].n_excl = ex.shape[0]
            self._sys[k].excl = ex.ctypes.data if ex.shape[0] else None
            for d in range(3):
                self._sys[k].box[d] = float(s.box[d])
        self._sig = np.ascontiguousarray(ff.sigma, np.float64)
        self._eps = np.ascontiguousarray(ff.epsilon, np.float64)
        self._chg = np.ascontiguousarray(ff.charge, np.float64)
        self._p = Params_t(self.n_types, self._sig.ctypes.data, self._eps.ctypes.data, self._chg.ctypes.data,
                           float(cutoff), float(skin), float(switch_width), float(dsf_alpha), float(sc_alpha),
                           self.schedule, self.precision, int(variant), float(capacity_factor),
                           int(electrostatics), int(pme_order), float(pme_spacing))
        self.electrostatics = int(electrostatics)
        self.ctx = None
        # bumped by every call that rewrites the forward state (list, slots,
        # force sums): a backward needs the state of its own forward
        self.generation = 0
        self._list_mode = LIST_AUTO
        self.static_scratch = bool(static_scratch)
        self._create()
        self.stream = torch.cuda.current_stream(self.device)
        self._bind()
        self.auto_capacity = auto_capacity

    # ------------------------------------------------------------ plumbing
    def _check(self, where, st):
        if st != 0:
            raise AlchNBError(where, st, self.lib.alch_nb_last_hip_error(self.ctx) if self.ctx else 0)

    def _create(self):
        ctx = ctypes.c_void_p()
        st = self.lib.alch_nb_create(ctypes.byref(self._p), self._sys, self.K, ctypes.byref(ctx))
        self._check("alch_nb_create", st)
        self.ctx = ctx
        nb = ctypes.c_size_t()
        self._check("alch_nb_workspace_size", self.lib.alch_nb_workspace_size(self.ctx, ctypes.byref(nb)))
        self.workspace_bytes = nb.value

    def pme_grid(self, k=0):
        """PME grid points (x, y, z) of box k."""
        dims = (ctypes.c_int32 * 3)()
        self._check("alch_nb_pme_grid", self.lib.alch_nb_pme_grid(self.ctx, int(k), dims))
        return tuple(int(v) for v in dims)

    def _bind(self):
        torch = self.torch
        if self.static_scratch:
            # the library's own device array: nothing is allocated here
            self.ws = None
            self._check("alch_nb_bind_static",
                        self.lib.alch_nb_bind_static(self.ctx, ctypes.c_void_p(self.stream.cuda_stream)))
            return
        self.ws = torch.empty(self.workspace_bytes + 256, dtype=torch.uint8, device=self.device)
        base = self.ws.data_ptr()
        aligned = (base + 255) & ~255
        self._check("alch_nb_bind", self.lib.alch_nb_bind(self.ctx, ctypes.c_void_p(aligned),
                                                          self.workspace_bytes, ctypes.c_void_p(self.stream.cuda_stream)))

    def grow_capacity(self, factor=2.0):
        """Re-plan with a larger list capacity (after FLAG_CAPACITY)."""
        self.lib.alch_nb_destroy(self.ctx)
        self._p.list_capacity_factor = max(1.0, self._p.list_capacity_factor) * factor
        self._create()
        self._bind()
        self.generation += 1
        if self._list_mode != LIST_AUTO:
            self.set_list_mode(self._list_mode)

    def set_list_mode(self, mode):
        """LIST_AUTO (fused build when co-resident) or LIST_PHASES (one kernel per phase)."""
        self._check("alch_nb_set_list_mode", self.lib.alch_nb_set_list_mode(self.ctx, int(mode)))
        self._list_mode = int(mode)

    def list_mode(self) -> int:
        """What a rebuild launches now: LIST_FUSED_ACTIVE or LIST_PHASES."""
        return int(self.lib.alch_nb_get_list_mode(self.ctx))

    def close(self):
        if self.ctx:
            self.lib.alch_nb_destroy(self.ctx)
            self.ctx = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    # ------------------------------------------------------------ tensors
    def positions(self, systems_or_array):
        """Concatenated float64 [N, 3] device tensor from systems or an array."""
        torch = self.torch
        if isinstance(systems_or_array, (list, tuple)):
            arr = np.concatenate([np.asarray(s.positions, np.float64) for s in systems_or_array])
        else:
            arr = np.asarray(systems_or_array, np.float64)
        return torch.as_tensor(arr.reshape(-1, 3), dtype=torch.float64, device=self.device).contiguous()

    def lambdas(self, lam):
        return self.torch.as_tensor(np.asarray(lam, np.float64).reshape(self.K), dtype=self.torch.float64,
                                    device=self.device).contiguous()

    def new_outputs(self, forces=True):
        torch = self.torch
        return dict(terms=torch.zeros((self.K, NTERMS), dtype=torch.float64, device=self.device),
                    forces=torch.zeros((self.N, 3), dtype=torch.float64, device=self.device) if forces else None,
                    dudl=torch.zeros(self.K, dtype=torch.float64, device=self.device),
                    n_pairs=torch.zeros(self.K, dtype=torch.int64, device=self.device))

    @staticmethod
    def _out_struct(out):
        return Out_t(_addr(out.get("terms")), _addr(out.get("forces")), _addr(out.get("dudl")),
                     _addr(out.get("n_pairs")))

    # ------------------------------------------------------------ calls
    def build_list(self, pos):
        self.generation += 1
        self._check("alch_nb_build_list", self.lib.alch_nb_build_list(self.ctx, ctypes.c_void_p(pos.data_ptr())))

    def compute(self, pos, lam, flags=AUTO_REBUILD, out=None):
        """Enqueue one evaluation; returns the output dict (device tensors)."""
        assert pos.dtype == self.torch.float64 and pos.is_contiguous() and pos.shape == (self.N, 3)
        assert lam.dtype == self.torch.float64 and lam.is_contiguous() and lam.shape == (self.K,)
        out = out if out is not None else self.new_outputs()
        self.generation += 1
        o = self._out_struct(out)
        self._out_keep = o
        st = self.lib.alch_nb_compute(self.ctx, ctypes.c_void_p(pos.data_ptr()), ctypes.c_void_p(lam.data_ptr()),
                                      int(flags), ctypes.byref(o))
        self._check("alch_nb_compute", st)
        return out

    def compute_checked(self, pos, lam, flags=AUTO_REBUILD, out=None, retries=3):
        """compute() that syncs and reads the flags: a fused list build whose
        barrier wait gave up is redone with one kernel per phase, and a list
        that outgrew its capacity is re-planned larger (when auto_capacity);
        either way the call is evaluated again with a forced rebuild.  The
        result carries the flags of the last evaluation."""
        for _ in range(retries + 1):
            res = self.compute(pos, lam, flags, out)
            f = self.get_flags()
            if f & FLAG_BARRIER_TIMEOUT and self._list_mode != LIST_PHASES:
                self.set_list_mode(LIST_PHASES)
                flags = FORCE_REBUILD
                continue
            if f & FLAG_CAPACITY and self.auto_capacity:
                self.grow_capacity()
                flags = FORCE_REBUILD
                continue
            res["flags"] = f
            return res
        raise AlchNBError("compute_checked", 4)

    def backward(self, pos, lam, grad_energy, d_pos=None, d_lambda=None, d_sigma=None, d_sqrt_eps=None,
                 d_charge=None, d_eps=None):
        g = Grad_t(_addr(d_pos), _addr(d_lambda), _addr(d_sigma), _addr(d_sqrt_eps), _addr(d_charge),
                   _addr(d_eps))
        st = self.lib.alch_nb_backward(self.ctx, ctypes.c_void_p(pos.data_ptr()), ctypes.c_void_p(lam.data_ptr()),
                                       ctypes.c_void_p(grad_energy.data_ptr()), ctypes.byref(g))
        self._check("alch_nb_backward", st)

    def dihedrals(self, pos, idx, mass_inv=None, s=None, kappa=None, forces=None, out=None):
        """Dihedral CVs; `out` (a dict returned by an earlier call with the same n and options) is
        reused instead of new zeroed outputs (a CV with an invalid index then keeps its old values)."""
        torch = self.torch
        n = int(idx.shape[0])
        if out is not None:
            xi, dxi, msum, u = out["xi"], out["dxi"], out["msum"], out["u_dafed"]
            assert xi.shape == (n,) and (msum is not None) == (mass_inv is not None)
            assert (u is not None) == (s is not None)
        else:
            xi = torch.zeros(n, dtype=torch.float64, device=self.device)
            dxi = torch.zeros((n, 4, 3), dtype=torch.float64, device=self.device)
            msum = torch.zeros(n, dtype=torch.float64, device=self.device) if mass_inv is not None else None
            u = torch.zeros(1, dtype=torch.float64, device=self.device) if s is not None else None
        st = self.lib.alch_nb_dihedrals(self.ctx, ctypes.c_void_p(pos.data_ptr()), n,
                                        ctypes.c_void_p(idx.data_ptr()), ctypes.c_void_p(xi.data_ptr()),
                                        ctypes.c_void_p(dxi.data_ptr()), _addr(mass_inv), _addr(msum), _addr(s),
                                        _addr(kappa), _addr(u), _addr(forces))
        self._check("alch_nb_dihedrals", st)
        return dict(xi=xi, dxi=dxi, msum=msum, u_dafed=u)

    def opes_state(self, capacity, kT, sigma=0.10, barrier_std=30.0, barrier_expl=5.0, theta0=0.0):
        """New device OPES state (float64) initialised on the bound stream."""
        n = int(self.lib.alch_nb_opes_state_size(int(capacity)))
        if n <= 0:
            raise AlchNBError("alch_nb_opes_state_size", 1)
        st = self.torch.empty(n, dtype=self.torch.float64, device=self.device)
        self._check("alch_nb_opes_init", self.lib.alch_nb_opes_init(self.ctx, ctypes.c_void_p(st.data_ptr()),
                                                                    int(capacity), float(kT), float(sigma),
                                                                    float(barrier_std), float(barrier_expl),
                                                                    float(theta0)))
        return st

    def opes_update(self, state, dudl, lam_out, deposit=False):
        st = self.lib.alch_nb_opes_update(self.ctx, ctypes.c_void_p(state.data_ptr()), _addr(dudl),
                                          _addr(lam_out), int(bool(deposit)))
        self._check("alch_nb_opes_update", st)

    # ------------------------------------------------------------ lambda dynamics
    def ld_init(self, params, theta0, s0=None, mass_s=None, kappa=None):
        """New lambda-dynamics state (device float64) for the context's K boxes.
        params: dict of alch_nb_ld_params fields.  Returns (state, layout dict)."""
        torch = self.torch
        q = LdParams_t(**params)
        n = int(self.lib.alch_nb_ld_state_size(ctypes.byref(q), self.K))
        if n <= 0:
            raise AlchNBError("alch_nb_ld_state_size", 1)
        off = (ctypes.c_int64 * len(LD_LAYOUT))()
        self._check("alch_nb_ld_layout", self.lib.alch_nb_ld_layout(ctypes.byref(q), self.K, off, len(LD_LAYOUT)))
        state = torch.empty(n, dtype=torch.float64, device=self.device)
        f64 = lambda a: None if a is None else torch.as_tensor(np.asarray(a, np.float64), dtype=torch.float64,
                                                              device=self.device).contiguous()
        th, s_, m_, k_ = f64(theta0), f64(s0), f64(mass_s), f64(kappa)
        self._ld_keep = (th, s_, m_, k_)
        self._check("alch_nb_ld_init", self.lib.alch_nb_ld_init(self.ctx, ctypes.byref(q), ctypes.c_void_p(state.data_ptr()),
                                                                _addr(th), _addr(s_), _addr(m_), _addr(k_)))
        lay = dict(zip(LD_LAYOUT, (int(v) for v in off)))
        lay.update(capacity=q.capacity, ti_bins=q.ti_bins, n_cv=q.n_cv, K=self.K)
        return state, lay

    def ld_step(self, state, dudl, noise, lam_out, xi=None):
        """One lambda-dynamics step; noise is a [rows, K + n_cv] float64 device tensor."""
        st = self.lib.alch_nb_ld_step(self.ctx, ctypes.c_void_p(state.data_ptr()), ctypes.c_void_p(dudl.data_ptr()),
                                      _addr(xi), ctypes.c_void_p(noise.data_ptr()), int(noise.shape[0]),
                                      _addr(lam_out))
        self._check("alch_nb_ld_step", st)

    def ld_step_dafed(self, state, dudl, noise, lam_out, pos, idx, xi=None, u_dafed=None, forces=None):
        """One lambda-dynamics step that also evaluates the d-AFED dihedral CVs (idx [n_cv, 4] int32) at
        pos in the same launch, with s and kappa from the state; the coupling force is added to `forces`."""
        st = self.lib.alch_nb_ld_step_dafed(self.ctx, ctypes.c_void_p(state.data_ptr()),
                                            ctypes.c_void_p(dudl.data_ptr()), ctypes.c_void_p(pos.data_ptr()),
                                            ctypes.c_void_p(idx.data_ptr()), _addr(xi), _addr(u_dafed),
                                            _addr(forces), ctypes.c_void_p(noise.data_ptr()), int(noise.shape[0]),
                                            _addr(lam_out))
        self._check("alch_nb_ld_step_dafed", st)

    def ld_free_energy(self, state):
        out = self.torch.empty(self.K, dtype=self.torch.float64, device=self.device)
        self._check("alch_nb_ld_free_energy", self.lib.alch_nb_ld_free_energy(
            self.ctx, ctypes.c_void_p(state.data_ptr()), ctypes.c_void_p(out.data_ptr())))
        return out

    @staticmethod
    def ld_view(state, lay):
        """Host copy of a lambda-dynamics state as per-replica dicts and the auxiliary arrays."""
        a = state.detach().cpu().numpy()
        cap, nb, K, ncv = lay["capacity"], lay["ti_bins"], lay["K"], lay["n_cv"]
        reps = []
        for r in range(K):
            b = lay["rep0"] + r * lay["rep_stride"]
            rec = {k: a[b + lay[k]] for k in ("theta", "p", "lambda", "last_lambda", "u_opes", "du_opes", "f_theta")}
            rec["n"] = int(a[b + lay["n"]])
            for name, key, cnt in (("std", "kern_std", "n_std"), ("expl", "kern_expl", "n_expl")):
                m = int(a[b + lay[cnt]])
                k0 = b + lay[key]
                rec[name] = (a[k0:k0 + m].copy(), a[k0 + cap:k0 + cap + m].copy(), a[k0 + 2 * cap:k0 + 2 * cap + m].copy())
            t0 = b + lay["ti"]
            rec["ti_sum"], rec["ti_cnt"] = a[t0:t0 + nb].copy(), a[t0 + nb:t0 + 2 * nb].copy()
            reps.append(rec)
        aux = dict(s=a[lay["cv_s"]:lay["cv_s"] + ncv].copy(), p=a[lay["cv_p"]:lay["cv_p"] + ncv].copy(),
                   force=a[lay["cv_force"]:lay["cv_force"] + ncv].copy())
        return reps, aux

    # ------------------------------------------------------------ replica exchange
    def hrex_init(self):
        """(state_of int32 [K], stats int64 [2K-1]) device tensors, identity assignment."""
        torch = self.torch
        so = torch.empty(self.K, dtype=torch.int32, device=self.device)
        stt = torch.empty(2 * self.K - 1, dtype=torch.int64, device=self.device)
        self._check("alch_nb_hrex_init", self.lib.alch_nb_hrex_init(self.ctx, ctypes.c_void_p(so.data_ptr()),
                                                                    ctypes.c_void_p(stt.data_ptr())))
        return so, stt

    def hrex_exchange(self, terms, lambda_states, state_of, lam, uniform, kT, stats):
        st = self.lib.alch_nb_hrex_exchange(self.ctx, ctypes.c_void_p(terms.data_ptr()),
                                            ctypes.c_void_p(lambda_states.data_ptr()),
                                            ctypes.c_void_p(state_of.data_ptr()), ctypes.c_void_p(lam.data_ptr()),
                                            ctypes.c_void_p(uniform.data_ptr()), int(uniform.shape[0]), float(kT),
                                            ctypes.c_void_p(stats.data_ptr()))
        self._check("alch_nb_hrex_exchange", st)

    def capture_begin(self):
        self._check("alch_nb_capture_begin", self.lib.alch_nb_capture_begin(self.ctx))

    def capture_end(self):
        self._check("alch_nb_capture_end", self.lib.alch_nb_capture_end(self.ctx))

    def export_pairs(self, cap=None):
        """Sorted int32 [m, 2] pair set of the current list (syncs)."""
        torch = self.torch
        n = ctypes.c_int64()
        cap = cap or max(1024, 400 * self.N)
        while True:
            buf = torch.empty((cap, 2), dtype=torch.int32, device=self.device)
            st = self.lib.alch_nb_export_pairs(self.ctx, ctypes.c_void_p(buf.data_ptr()), cap, ctypes.byref(n))
            if st == 4:
                cap = int(n.value) + 1
                continue
            self._check("alch_nb_export_pairs", st)
            break
        arr = buf[: n.value].cpu().numpy()
        order = np.lexsort((arr[:, 1], arr[:, 0]))
        return arr[order]

    def capture_step(self, pos, lam, out):
        o = self._out_struct(out)
        self._graph_out = o
        self._graph_keep = (pos, lam, out)
        st = self.lib.alch_nb_capture_step(self.ctx, ctypes.c_void_p(pos.data_ptr()),
                                           ctypes.c_void_p(lam.data_ptr()), ctypes.byref(o))
        self._check("alch_nb_capture_step", st)

    def launch_step(self):
        self._check("alch_nb_launch_step", self.lib.alch_nb_launch_step(self.ctx))

    def autotune(self, pos, lam, reps=5):
        self.generation += 1
        self._check("alch_nb_autotune", self.lib.alch_nb_autotune(self.ctx, ctypes.c_void_p(pos.data_ptr()),
                                                                  ctypes.c_void_p(lam.data_ptr()), int(reps)))

    def set_variant(self, v):
        self.generation += 1
        self._check("alch_nb_set_variant", self.lib.alch_nb_set_variant(self.ctx, int(v)))

    def set_timing(self, on=True, every=1):
        """Time the tile launch of every `every`-th call from now on (off: on=False)."""
        self._check("alch_nb_set_timing", self.lib.alch_nb_set_timing(self.ctx, int(every) if on else 0))

    def get_flags(self) -> int:
        f = ctypes.c_uint32()
        self._check("alch_nb_get_flags", self.lib.alch_nb_get_flags(self.ctx, ctypes.byref(f)))
        return int(f.value)

    def get_stats(self) -> dict:
        s = Stats_t()
        self._check("alch_nb_get_stats", self.lib.alch_nb_get_stats(self.ctx, ctypes.byref(s)))
        return {name: getattr(s, name) for name, _ in Stats_t._fields_}


def flops_per_pair(kind: int) -> float:
    return float(load().alch_nb_flops_per_pair(int(kind)))


def from_workload(w, precision=FP32_FIXED, schedule=BEUTLER_DSF, **kw) -> Context:
    return Context(w.ff, w.systems, w.cutoff, w.skin, w.switch_width, w.dsf_alpha, w.sc_alpha, schedule=schedule,
                   precision=precision, **kw)
