"""Thin ctypes binding of libugkwp.so (the C ABI in include/ugkwp.h).

Argument marshalling only: every step of the UGKWP time step runs in the HIP
kernels of the library.  There is no CPU fallback; loading fails loudly when
the library has not been built.
"""
from __future__ import annotations

import ctypes as C
import os
from typing import Optional, Sequence

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libugkwp.so")

OK, EINVAL, ENOMEM, EPOOL, ENOCONV, ENONFINITE, EHIP = 0, -1, -2, -3, -4, -5, -6
BC_VACUUM, BC_PLANCK, BC_REFLECT = 0, 1, 2
FLAG_GROUP_SIGMA = 1
FLAG_GRAPH = 2
FLAG_PHASE_TIMES = 4
FLAG_SI_LINEARIZED = 8
FLAG_SLOPES = 16
FLAG_WAVE_ITER = 32
FLAG_BOUNDARY_PARTICLES = 64
PURPOSE_BIRTH, PURPOSE_FLIGHT = 1, 2

EXPORTED = [
    "ugkwp_create", "ugkwp_destroy", "ugkwp_last_error", "ugkwp_init_mesh", "ugkwp_set_opacity",
    "ugkwp_set_material", "ugkwp_init_batch", "ugkwp_step", "ugkwp_num_instances",
    "ugkwp_get_fields", "ugkwp_get_tallies", "ugkwp_get_diag", "ugkwp_get_counters",
    "ugkwp_pool_size", "ugkwp_get_pool", "ugkwp_set_pool", "ugkwp_eval_phi", "ugkwp_eval_coef",
    "ugkwp_eval_uniform", "ugkwp_eval_neg_log", "ugkwp_eval_sample_nu", "ugkwp_record", "ugkwp_recorded_steps",
    "ugkwp_adjoint", "ugkwp_autotune", "ugkwp_get_totals", "ugkwp_set_phase_times", "ugkwp_set_push_timing",
    "ugkwp_state_bytes", "ugkwp_get_state", "ugkwp_set_state", "ugkwp_set_material_noalloc",
    "ugkwp_set_heat_capacity", "ugkwp_set_source", "ugkwp_set_source_planck", "ugkwp_set_opacity_table",
]

_d = C.c_double
_pd = C.POINTER(C.c_double)
_pu64 = C.POINTER(C.c_uint64)
_pi64 = C.POINTER(C.c_int64)
_pi32 = C.POINTER(C.c_int32)
_pu32 = C.POINTER(C.c_uint32)
_pu8 = C.POINTER(C.c_uint8)
_pint = C.POINTER(C.c_int)


class Params(C.Structure):
    _fields_ = [("c", _d), ("a", _d), ("eps", _d), ("dt", _d), ("nu_power", _d),
                ("n_cap", C.c_int64), ("pool_capacity", C.c_int64), ("si_max_iters", C.c_int),
                ("si_tol", _d), ("flags", C.c_uint32), ("sort_interval", C.c_int),
                ("tau_num_C", _d), ("tau_num_jump", _d), ("opacity_T_power", _d),
                ("opacity_stim", C.c_int32)]


class Instance(C.Structure):
    _fields_ = [("dim", C.c_int), ("nx", C.c_int), ("ny", C.c_int),
                ("x0", _d), ("x1", _d), ("y0", _d), ("y1", _d),
                ("bc", C.c_int * 4), ("bcT", _d * 4), ("G", C.c_int), ("nu_edges", _pd),
                ("seed", C.c_uint64), ("w_ref", _d), ("kappa", _pd), ("cv", _pd), ("T0", _pd),
                ("Tr0", _pd), ("pinned", _pu8)]


class AdjointStats(C.Structure):
    _fields_ = [("steps", C.c_int), ("sweeps_launched", C.c_int), ("sweeps_max", C.c_int), ("ms", _d),
                ("ms_sweeps", _d), ("cell_group_updates", C.c_longlong)]

    def as_dict(self):
        return {k: getattr(self, k) for k, _ in self._fields_}


class Totals(C.Structure):
    _fields_ = [("steps", C.c_int64), ("n_pushed", C.c_int64), ("n_survived", C.c_int64),
                ("sweeps_max", C.c_int64), ("sweeps_sum", C.c_int64), ("ms_sample", _d), ("ms_push", _d),
                ("ms_macro", _d), ("ms_si", _d), ("ms_sort", _d), ("cg_updates", C.c_int64),
                ("push_timed", C.c_int64), ("n_pushed_timed", C.c_int64), ("n_survived_timed", C.c_int64)]

    def as_dict(self):
        return {k: getattr(self, k) for k, _ in self._fields_}


class TuneResult(C.Structure):
    _fields_ = [("ppt", C.c_int), ("blocks", C.c_int), ("candidates", C.c_int), ("us_best", _d),
                ("us_default", _d), ("threads", C.c_int)]

    def as_dict(self):
        return {k: getattr(self, k) for k, _ in self._fields_}


class Diag(C.Structure):
    _fields_ = [("n_alive_in", C.c_int64), ("n_births", C.c_int64), ("n_alive_out", C.c_int64),
                ("n_pushed", C.c_int64), ("sweeps_max", C.c_int), ("sweeps_sum", C.c_int),
                ("e_start", _d), ("e_end", _d), ("inflow_wave", _d), ("inflow_eq", _d),
                ("exit_particles", _d), ("injection", _d), ("residual", _d),
                ("ms_sample", _d), ("ms_push", _d), ("ms_macro", _d), ("ms_si", _d), ("ms_sort", _d),
                ("push_timed", C.c_int), ("inflow_particles", _d)]

    def as_dict(self):
        return {k: getattr(self, k) for k, _ in self._fields_}


_lib = None


def load():
    """Load libugkwp.so; raises if it is missing (no fallback path exists)."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH):
        raise RuntimeError(f"{LIB_PATH} is not built: run __graft_entry__.build() or "
                           "python paper_2312_16981_amd/build.py")
    # PyTorch-ROCm ships its own HIP runtime under the same soname.  Loading it
    # first makes the library bind to that one copy, so that torch streams and
    # device pointers can be handed to the library; a second copy loaded after
    # the system runtime leaves torch without a device.
    try:
        import torch  # noqa: F401
    except ImportError:
        pass
    L = C.CDLL(LIB_PATH)
    vp = C.c_void_p
    L.ugkwp_create.argtypes = [C.POINTER(vp), C.POINTER(Params), vp]
    L.ugkwp_destroy.argtypes = [vp]
    L.ugkwp_destroy.restype = None
    L.ugkwp_last_error.argtypes = [vp]
    L.ugkwp_last_error.restype = C.c_char_p
    L.ugkwp_init_mesh.argtypes = [vp, C.c_int, C.c_int, C.c_int, _pd, _pd, _pint, _pd, C.c_int, _pd,
                                  C.c_uint64, _d]
    L.ugkwp_set_opacity.argtypes = [vp, _pd]
    L.ugkwp_set_material.argtypes = [vp, _pd, _pd, _pd, _pu8]
    L.ugkwp_set_material_noalloc.argtypes = [vp, _pd, _pd, _pd, _pu8]
    L.ugkwp_init_batch.argtypes = [vp, C.c_int, C.POINTER(Instance)]
    L.ugkwp_set_heat_capacity.argtypes = [vp, _pd, _pd]
    L.ugkwp_set_source.argtypes = [vp, _pd, _d]
    L.ugkwp_set_source_planck.argtypes = [vp, _pd, _d, _d]
    L.ugkwp_set_opacity_table.argtypes = [vp, C.c_int, _pi32, C.c_int, _pd, C.c_int, _pd, _pd]
    L.ugkwp_step.argtypes = [vp, C.c_int]
    L.ugkwp_num_instances.argtypes = [vp]
    L.ugkwp_get_fields.argtypes = [vp, C.c_int, _pd, _pd, _pd, C.c_int]
    L.ugkwp_get_tallies.argtypes = [vp, C.c_int, _pd, _pd, _pd, _pd, _pi64, _pd, _pd]
    L.ugkwp_get_diag.argtypes = [vp, C.POINTER(Diag)]
    L.ugkwp_get_counters.argtypes = [vp, C.c_int, _pu64, _pint]
    L.ugkwp_pool_size.argtypes = [vp]
    L.ugkwp_pool_size.restype = C.c_int64
    L.ugkwp_get_pool.argtypes = [vp, _pd, _pd, _pd, _pd, _pd, _pd, _pu64, _pi32, _pi32]
    L.ugkwp_set_pool.argtypes = [vp, C.c_int64, _pd, _pd, _pd, _pd, _pd, _pd, _pu64, _pi32, _pi32,
                                 C.c_uint64, _pd]
    L.ugkwp_state_bytes.argtypes = [vp]
    L.ugkwp_state_bytes.restype = C.c_int64
    L.ugkwp_get_state.argtypes = [vp, vp, C.c_int64]
    L.ugkwp_set_state.argtypes = [vp, vp, C.c_int64]
    L.ugkwp_record.argtypes = [vp, C.c_int]
    L.ugkwp_autotune.argtypes = [vp, C.POINTER(TuneResult)]
    L.ugkwp_get_totals.argtypes = [vp, C.POINTER(Totals), C.c_int]
    L.ugkwp_set_phase_times.argtypes = [vp, C.c_int]
    L.ugkwp_set_push_timing.argtypes = [vp, C.c_int]
    L.ugkwp_recorded_steps.argtypes = [vp]
    L.ugkwp_adjoint.argtypes = [vp, _pd, _pd, C.c_int, C.POINTER(AdjointStats)]
    L.ugkwp_eval_phi.argtypes = [C.c_int, _pd, C.c_int, _pd, _d, _d, _pd]
    L.ugkwp_eval_coef.argtypes = [C.c_int, _pd, _pd, _pd, _pd]
    L.ugkwp_eval_uniform.argtypes = [C.c_int, C.c_uint64, _pu64, C.c_uint32, C.c_uint32, _pu32, _pd]
    L.ugkwp_eval_neg_log.argtypes = [C.c_int, _pd, _pd]
    L.ugkwp_eval_sample_nu.argtypes = [C.c_int, _pd, _pd, _pd, _pd, _pd, _pd]
    _lib = L
    return L


def _p(a, t=_pd):
    return None if a is None else a.ctypes.data_as(t)


class UGKWPError(RuntimeError):
    def __init__(self, code, msg):
        super().__init__(f"ugkwp error {code}: {msg}")
        self.code = code


def _f64(a):
    return np.ascontiguousarray(a, dtype=np.float64)


class Context:
    """One library context: a single instance (init_mesh / set_opacity /
    set_material) or a batch of independent instances (init_batch)."""

    def __init__(self, params: Params, stream=None):
        L = load()
        h = C.c_void_p()
        st = C.c_void_p(stream) if stream else None
        rc = L.ugkwp_create(C.byref(h), C.byref(params), st)
        if rc:
            raise UGKWPError(rc, "create")
        self.h = h
        self.params = params
        self.layout = []          # (ncell, G, nx, ny, dim) per instance
        self._keep = []

    def _chk(self, rc, what):
        if rc:
            raise UGKWPError(rc, f"{what}: {load().ugkwp_last_error(self.h).decode()}")
        return rc

    def close(self):
        if getattr(self, "h", None):
            load().ugkwp_destroy(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    # ---- set-up (same names as the C ABI) ----
    def init_mesh(self, dim, nx, ny, lo, hi, bc, bcT, nu_edges, seed, w_ref):
        L = load()
        lo_a, hi_a = _f64(lo), _f64(hi)
        bc_a = (C.c_int * 4)(*[int(b) for b in bc])
        bcT_a = _f64(bcT)
        nu = _f64(nu_edges)
        self._chk(L.ugkwp_init_mesh(self.h, dim, nx, ny, _p(lo_a), _p(hi_a), bc_a, _p(bcT_a),
                                    len(nu) - 1, _p(nu), int(seed), float(w_ref)), "init_mesh")
        self.layout = [(nx * ny, len(nu) - 1, nx, ny, dim)]

    def set_opacity(self, kappa):
        k = _f64(kappa)
        self._chk(load().ugkwp_set_opacity(self.h, _p(k)), "set_opacity")

    def set_material(self, cv, T0, Tr0, pinned=None):
        a, b, c = _f64(cv), _f64(T0), _f64(Tr0)
        p = None if pinned is None else np.ascontiguousarray(pinned, dtype=np.uint8)
        self._chk(load().ugkwp_set_material(self.h, _p(a), _p(b), _p(c), _p(p, _pu8)), "set_material")

    def set_material_noalloc(self, cv, T0, Tr0, pinned=None):
        """set_material without device allocation (static per-GPU staging; see ugkwp.h)."""
        a, b, c = _f64(cv), _f64(T0), _f64(Tr0)
        p = None if pinned is None else np.ascontiguousarray(pinned, dtype=np.uint8)
        self._chk(load().ugkwp_set_material_noalloc(self.h, _p(a), _p(b), _p(c), _p(p, _pu8)),
                  "set_material_noalloc")

    def set_heat_capacity(self, H, chi):
        """Olson's heat capacity per cell (H = 0: the cell keeps its C_v); H None: off."""
        if H is None:
            self._chk(load().ugkwp_set_heat_capacity(self.h, None, None), "set_heat_capacity")
            return
        a, b = _f64(H), _f64(chi)
        self._chk(load().ugkwp_set_heat_capacity(self.h, _p(a), _p(b)), "set_heat_capacity")

    def set_source(self, q, t_off=float("inf")):
        """Volumetric source rate q [ncell][G]; None: off."""
        a = None if q is None else _f64(q)
        self._chk(load().ugkwp_set_source(self.h, _p(a), float(t_off)), "set_source")

    def set_source_planck(self, f, Ts, t_off=float("inf")):
        """The source B(nu, Ts) f(x) (rate (c/eps^2) f phi_g(Ts), computed on the device)."""
        a = _f64(f)
        self._chk(load().ugkwp_set_source_planck(self.h, _p(a), float(Ts), float(t_off)), "set_source_planck")

    def set_opacity_table(self, mat, nu, T, sigma):
        """Tabulated sigma [nmat][nT][nnu] on nodes nu, T; mat [ncell]."""
        m = np.ascontiguousarray(mat, dtype=np.int32)
        n, t, sg = _f64(nu), _f64(T), _f64(sigma)
        self._chk(load().ugkwp_set_opacity_table(self.h, int(sg.shape[0]), _p(m, _pi32), len(n), _p(n), len(t),
                                                 _p(t), _p(sg)), "set_opacity_table")

    def init_batch(self, instances: Sequence["Instance"], arrays_keepalive):
        arr = (Instance * len(instances))(*instances)
        self._chk(load().ugkwp_init_batch(self.h, len(instances), arr), "init_batch")

    def step(self, n=1, check=True):
        rc = load().ugkwp_step(self.h, n)
        if check:
            self._chk(rc, "step")
        return rc

    def autotune(self):
        """Pick the push launch shape by timing it on the current pool (see ugkwp.h)."""
        r = TuneResult()
        self._chk(load().ugkwp_autotune(self.h, C.byref(r)), "autotune")
        return r.as_dict()

    # ---- adjoint of the frozen-tally macroscopic map ----
    def record(self, max_steps):
        """Keep a record of up to max_steps following steps (0 stops and frees it)."""
        self._chk(load().ugkwp_record(self.h, int(max_steps)), "record")

    def recorded_steps(self):
        return int(load().ugkwp_recorded_steps(self.h))

    def adjoint(self, dJdT):
        """dJ/dkappa [all cells][G] (instances concatenated) of J = sum dJdT * T(final)."""
        d = _f64(dJdT).reshape(-1)
        if d.size != sum(n for n, *_ in self.layout):
            raise ValueError("dJdT needs one value per cell of every instance")
        total = sum(n * g for n, g, *_ in self.layout)
        out = np.zeros(total)
        st = AdjointStats()
        self._chk(load().ugkwp_adjoint(self.h, _p(d), _p(out), 0, C.byref(st)), "adjoint")
        self.last_adjoint = st.as_dict()
        return out

    def adjoint_device(self, dJdT_ptr, grad_ptr):
        """Device-pointer variant (e.g. torch tensors' data_ptr()), on the context stream."""
        st = AdjointStats()
        self._chk(load().ugkwp_adjoint(self.h, C.cast(dJdT_ptr, _pd), C.cast(grad_ptr, _pd), 1,
                                       C.byref(st)), "adjoint")
        self.last_adjoint = st.as_dict()
        return self.last_adjoint

    # ---- results ----
    def get_fields(self, inst=0):
        ncell, G = self.layout[inst][0], self.layout[inst][1]
        rho = np.zeros((ncell, G))
        T = np.zeros(ncell)
        rhop = np.zeros((ncell, G))
        self._chk(load().ugkwp_get_fields(self.h, inst, _p(rho), _p(T), _p(rhop), 0), "get_fields")
        return rho, T, rhop

    def get_fields_device(self, rho_ptr, T_ptr, inst=-1):
        """Write fields into device buffers (e.g. torch tensors' data_ptr())."""
        self._chk(load().ugkwp_get_fields(self.h, inst, C.cast(rho_ptr, _pd) if rho_ptr else None,
                                          C.cast(T_ptr, _pd) if T_ptr else None, None, 1), "get_fields")

    def get_tallies(self, inst=0):
        ncell, G, nx, ny, dim = self.layout[inst]
        fx = np.zeros(((nx + 1) * ny, G, 2))
        fy = np.zeros((nx * (ny + 1), G, 2)) if dim == 2 else None
        dep = np.zeros((ncell, G))
        surv = np.zeros((ncell, G))
        nb = np.zeros((ncell, G), np.int64)
        wnew = np.zeros((ncell, G))
        Q = np.zeros((ncell, G))
        self._chk(load().ugkwp_get_tallies(self.h, inst, _p(fx), _p(fy), _p(dep), _p(surv),
                                           _p(nb, _pi64), _p(wnew), _p(Q)), "get_tallies")
        return dict(fx=fx, fy=fy, dep=dep, surv=surv, nbirth=nb, wnew=wnew, Q=Q)

    def get_diag(self):
        d = Diag()
        self._chk(load().ugkwp_get_diag(self.h, C.byref(d)), "get_diag")
        return d.as_dict()

    def get_totals(self, reset=False):
        """Running sums over committed steps since the last reset (see ugkwp.h)."""
        t = Totals()
        self._chk(load().ugkwp_get_totals(self.h, C.byref(t), 1 if reset else 0), "get_totals")
        return t.as_dict()

    def set_phase_times(self, on=True):
        self._chk(load().ugkwp_set_phase_times(self.h, 1 if on else 0), "set_phase_times")

    def set_push_timing(self, every):
        self._chk(load().ugkwp_set_push_timing(self.h, int(every)), "set_push_timing")

    def get_counters(self, inst=0):
        b = C.c_uint64()
        s = C.c_int()
        self._chk(load().ugkwp_get_counters(self.h, inst, C.byref(b), C.byref(s)), "get_counters")
        return int(b.value), int(s.value)

    def pool_size(self):
        return int(load().ugkwp_pool_size(self.h))

    def get_pool(self):
        n = self.pool_size()
        out = dict(x=np.zeros(n), y=np.zeros(n), ox=np.zeros(n), oy=np.zeros(n), nu=np.zeros(n),
                   w=np.zeros(n), id=np.zeros(n, np.uint64), cell=np.zeros(n, np.int32),
                   g=np.zeros(n, np.int32))
        self._chk(load().ugkwp_get_pool(self.h, _p(out["x"]), _p(out["y"]), _p(out["ox"]), _p(out["oy"]),
                                        _p(out["nu"]), _p(out["w"]), _p(out["id"], _pu64),
                                        _p(out["cell"], _pi32), _p(out["g"], _pi32)), "get_pool")
        return out

    def set_pool(self, pool, birth_counter, rhop=None):
        n = len(pool["x"])
        a = {k: np.ascontiguousarray(v) for k, v in pool.items()}
        y = _f64(a["y"]) if "y" in a else None
        oy = _f64(a["oy"]) if "oy" in a else None
        self._chk(load().ugkwp_set_pool(self.h, n, _p(_f64(a["x"])), _p(y), _p(_f64(a["ox"])), _p(oy),
                                        _p(_f64(a["nu"])), _p(_f64(a["w"])),
                                        _p(a["id"].astype(np.uint64), _pu64),
                                        _p(a["cell"].astype(np.int32), _pi32),
                                        _p(a["g"].astype(np.int32), _pi32), int(birth_counter),
                                        _p(_f64(rhop)) if rhop is not None else None), "set_pool")

    def get_state(self):
        """The committed state as a byte array (ugkwp_get_state)."""
        n = load().ugkwp_state_bytes(self.h)
        self._chk(n if n < 0 else 0, "state_bytes")
        buf = np.zeros(n, np.uint8)
        self._chk(load().ugkwp_get_state(self.h, buf.ctypes.data, n), "get_state")
        return buf

    def set_state(self, buf):
        b = np.ascontiguousarray(buf, dtype=np.uint8)
        self._chk(load().ugkwp_set_state(self.h, b.ctypes.data, b.size), "set_state")


def make_params(c=1.0, a=1.0, eps=1.0, dt=1e-3, nu_power=3.0, n_cap=1 << 20, pool_capacity=1 << 20,
                si_max_iters=200, si_tol=1e-13, flags=0, sort_interval=0, tau_num_C=0.0,
                tau_num_jump=10.0, opacity_T_power=0.0, opacity_stim=0) -> Params:
    p = Params()
    p.sort_interval = sort_interval
    p.tau_num_C, p.tau_num_jump = tau_num_C, tau_num_jump
    p.opacity_T_power = opacity_T_power
    p.opacity_stim = opacity_stim
    p.c, p.a, p.eps, p.dt, p.nu_power = c, a, eps, dt, nu_power
    p.n_cap, p.pool_capacity, p.si_max_iters, p.si_tol, p.flags = n_cap, pool_capacity, si_max_iters, si_tol, flags
    return p


def from_problem(prob, stream=None, pool_capacity: Optional[int] = None, sort_interval: int = 0,
                 extra_flags: int = 0) -> Context:
    """Build a single-instance context from a workloads.Problem."""
    P = make_params(c=prob.c, a=prob.a, eps=prob.eps, dt=prob.dt, nu_power=prob.nu_power,
                    n_cap=prob.n_cap, pool_capacity=pool_capacity or prob.pool_cap,
                    si_max_iters=prob.si_max_iters, si_tol=prob.si_tol, flags=prob.flags | extra_flags,
                    sort_interval=sort_interval, tau_num_C=prob.tau_num_C, tau_num_jump=prob.tau_num_jump,
                    opacity_T_power=prob.T_power, opacity_stim=prob.opacity_stim)
    ctx = Context(P, stream)
    ctx.init_mesh(prob.dim, prob.nx, prob.ny, [prob.x0, prob.y0], [prob.x1, prob.y1], prob.bc, prob.bcT,
                  prob.nu_edges, prob.seed, prob.w_ref)
    ctx.set_opacity(prob.kappa)
    ctx.set_material(prob.cv, prob.T0, prob.Tr0, prob.pinned)
    _set_models(ctx, [prob])
    return ctx


def _set_models(ctx, probs):
    """Olson's material models of the problems (heat capacity, source, opacity
    table), concatenated over the instances: instances without a model get its
    neutral value (H = 0, q = 0, their own material numbers after the others')."""
    if any(p.olson_H is not None for p in probs):
        H = np.concatenate([np.zeros(p.ncell) if p.olson_H is None else np.asarray(p.olson_H, float) for p in probs])
        chi = np.concatenate([np.zeros(p.ncell) if p.olson_chi is None else np.asarray(p.olson_chi, float)
                              for p in probs])
        ctx.set_heat_capacity(H, chi)
    srcs = [p for p in probs if p.source is not None or p.source_shape is not None]
    if srcs:
        if len({p.source_t_off for p in srcs}) != 1:
            raise ValueError("the instances' sources must share their switch-off time")
        t_off = srcs[0].source_t_off
        if all(p.source is None for p in probs) and len({p.source_T for p in srcs}) == 1:
            f = np.concatenate([np.zeros(p.ncell) if p.source_shape is None else np.asarray(p.source_shape, float)
                                for p in probs])
            ctx.set_source_planck(f, srcs[0].source_T, t_off)
        elif all(p.source_shape is None for p in probs):
            ctx.set_source(np.concatenate([np.zeros(p.ncell * p.G) if p.source is None
                                           else np.asarray(p.source, float).reshape(-1) for p in probs]), t_off)
        else:
            raise ValueError("a batch takes either rate sources or Planckian sources of one temperature")
    tabs = [p.opacity_table for p in probs if p.opacity_table is not None]
    if tabs:
        if len(tabs) != len(probs):
            raise ValueError("a tabulated opacity must be given for every instance of a batch or none")
        t0 = tabs[0]
        if any(not (np.array_equal(t["nu"], t0["nu"]) and np.array_equal(t["T"], t0["T"])) for t in tabs):
            raise ValueError("the instances' opacity tables must share their nodes")
        mats, sig, off = [], [], 0
        for t in tabs:
            mats.append(np.asarray(t["mat"], np.int64) + off)
            sig.append(np.asarray(t["sigma"], float))
            off += sig[-1].shape[0]
        ctx.set_opacity_table(np.concatenate(mats), t0["nu"], t0["T"], np.concatenate(sig, axis=0))


def from_batch(probs, stream=None, pool_capacity: Optional[int] = None, sort_interval: int = 0,
               extra_flags: int = 0) -> Context:
    """Build a batched context from a list of workloads.Problem.  The parameters
    a context shares (dimension, c, a, eps, dt, opacity law, flags, iteration
    limits, tau_num) must agree across the list: ValueError otherwise."""
    p0 = probs[0]
    shared = ("dim", "c", "a", "eps", "dt", "nu_power", "n_cap", "si_max_iters", "si_tol", "flags",
              "tau_num_C", "tau_num_jump", "T_power", "opacity_stim")
    for k, pr in enumerate(probs):
        diff = [f for f in shared if getattr(pr, f) != getattr(p0, f)]
        if diff:
            raise ValueError(f"instance {k} differs from instance 0 in the shared parameters {diff}")
    cap = pool_capacity or sum(p.pool_cap for p in probs)
    P = make_params(c=p0.c, a=p0.a, eps=p0.eps, dt=p0.dt, nu_power=p0.nu_power, n_cap=p0.n_cap,
                    pool_capacity=cap, si_max_iters=p0.si_max_iters, si_tol=p0.si_tol,
                    flags=p0.flags | extra_flags, sort_interval=sort_interval, tau_num_C=p0.tau_num_C,
                    tau_num_jump=p0.tau_num_jump, opacity_T_power=p0.T_power,
                    opacity_stim=p0.opacity_stim)
    ctx = Context(P, stream)
    keep = []
    insts = []
    for pr in probs:
        arrs = dict(nu=_f64(pr.nu_edges), kappa=_f64(pr.kappa), cv=_f64(pr.cv), T0=_f64(pr.T0),
                    Tr0=_f64(pr.Tr0), pinned=np.ascontiguousarray(pr.pinned, dtype=np.uint8))
        keep.append(arrs)
        s = Instance()
        s.dim, s.nx, s.ny = pr.dim, pr.nx, pr.ny
        s.x0, s.x1, s.y0, s.y1 = pr.x0, pr.x1, pr.y0, pr.y1
        for q in range(4):
            s.bc[q] = int(pr.bc[q])
            s.bcT[q] = float(pr.bcT[q])
        s.G = pr.G
        s.nu_edges = _p(arrs["nu"])
        s.seed = int(pr.seed)
        s.w_ref = float(pr.w_ref)
        s.kappa, s.cv, s.T0, s.Tr0 = _p(arrs["kappa"]), _p(arrs["cv"]), _p(arrs["T0"]), _p(arrs["Tr0"])
        s.pinned = _p(arrs["pinned"], _pu8)
        insts.append(s)
    ctx.init_batch(insts, keep)
    ctx.layout = [(p.ncell, p.G, p.nx, p.ny, p.dim) for p in probs]
    ctx._keep = keep
    _set_models(ctx, probs)
    return ctx


# ---- element-wise device building blocks ----

def eval_phi(T, nu_edges, a=1.0, c=1.0):
    T = _f64(T)
    nu = _f64(nu_edges)
    out = np.zeros((len(T), len(nu) - 1))
    rc = load().ugkwp_eval_phi(len(T), _p(T), len(nu) - 1, _p(nu), a, c, _p(out))
    if rc:
        raise UGKWPError(rc, "eval_phi")
    return out


def eval_coef(s):
    s = _f64(s)
    c4, w, c2 = np.zeros_like(s), np.zeros_like(s), np.zeros_like(s)
    rc = load().ugkwp_eval_coef(len(s), _p(s), _p(c4), _p(w), _p(c2))
    if rc:
        raise UGKWPError(rc, "eval_coef")
    return c4, w, c2


def eval_uniform(seed, ids, step, purpose, d):
    ids = np.ascontiguousarray(ids, dtype=np.uint64)
    d = np.ascontiguousarray(d, dtype=np.uint32)
    out = np.zeros(len(ids))
    rc = load().ugkwp_eval_uniform(len(ids), int(seed), _p(ids, _pu64), step, purpose, _p(d, _pu32), _p(out))
    if rc:
        raise UGKWPError(rc, "eval_uniform")
    return out


def eval_neg_log(u):
    u = _f64(u)
    out = np.zeros_like(u)
    rc = load().ugkwp_eval_neg_log(len(u), _p(u), _p(out))
    if rc:
        raise UGKWPError(rc, "eval_neg_log")
    return out


def eval_sample_nu(nl, nh, T, U):
    nl, nh, T, U = _f64(nl), _f64(nh), _f64(T), _f64(U)
    beta, nu = np.zeros_like(nl), np.zeros_like(nl)
    rc = load().ugkwp_eval_sample_nu(len(nl), _p(nl), _p(nh), _p(T), _p(U), _p(beta), _p(nu))
    if rc:
        raise UGKWPError(rc, "eval_sample_nu")
    return beta, nu
