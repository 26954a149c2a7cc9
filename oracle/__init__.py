"""ctypes front end of the FP64 CPU oracle (liboracle.so).

TEST INFRASTRUCTURE ONLY: the tests, the smoke check and the benchmark's
CPU-baseline leg use it to check the GPU library.  It shares no code with
the GPU library and never imports it.
"""
from __future__ import annotations

import ctypes as C
import os

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
# UGKWP_ORACLE_LIB: another build of the same sources (e.g. the sanitized one
# that `python oracle/build.py --sanitize` makes)
_LIB = os.environ.get("UGKWP_ORACLE_LIB") or os.path.join(_HERE, "liboracle.so")
_lib = None

OK, EINVAL, ENOMEM, EPOOL, ENOCONV, ENONFINITE = 0, -1, -2, -3, -4, -5
PURPOSE_BIRTH, PURPOSE_FLIGHT = 1, 2

_d = C.c_double
_pd = C.POINTER(C.c_double)
_pu64 = C.POINTER(C.c_uint64)
_pi64 = C.POINTER(C.c_int64)
_pi32 = C.POINTER(C.c_int32)
_pu8 = C.POINTER(C.c_uint8)


class Params(C.Structure):
    _fields_ = [("dim", C.c_int), ("nx", C.c_int), ("ny", C.c_int),
                ("x0", _d), ("x1", _d), ("y0", _d), ("y1", _d),
                ("bc", C.c_int * 4), ("bcT", _d * 4),
                ("G", C.c_int), ("nu", _pd), ("nu_power", _d),
                ("c", _d), ("a", _d), ("eps", _d), ("dt", _d), ("w_ref", _d),
                ("n_cap", C.c_int64), ("seed", C.c_uint64), ("pool_cap", C.c_int64),
                ("si_max_iters", C.c_int), ("si_tol", _d), ("flags", C.c_int),
                ("tau_num_C", _d), ("tau_num_jump", _d), ("T_power", _d),
                ("opacity_stim", C.c_int)]


class Diag(C.Structure):
    _fields_ = [("n_alive_in", C.c_int64), ("n_births", C.c_int64), ("n_alive_out", C.c_int64),
                ("n_collided", C.c_int64), ("n_exited", C.c_int64), ("n_crossings", C.c_int64),
                ("sweeps", C.c_int),
                ("e_start", _d), ("e_end", _d), ("inflow_wave", _d), ("inflow_eq", _d),
                ("exit_particles", _d), ("injection", _d), ("residual", _d),
                ("si_drho", _d), ("si_rho", _d), ("si_dT", _d), ("si_T", _d),
                ("inflow_particles", _d), ("n_ghost_births", C.c_int64), ("n_ghost_entered", C.c_int64)]

    def as_dict(self):
        return {k: getattr(self, k) for k, _ in self._fields_}


def lib():
    global _lib
    if _lib is None:
        if not os.path.exists(_LIB):
            from . import build as _b
            _b.build()
        L = C.CDLL(_LIB)
        L.ora_philox4x32_10.argtypes = [C.POINTER(C.c_uint32), C.POINTER(C.c_uint32), C.POINTER(C.c_uint32)]
        L.ora_uniform.argtypes = [C.c_uint64, C.c_uint64, C.c_uint32, C.c_uint32, C.c_uint32]
        L.ora_uniform.restype = _d
        for f in ("ora_planck_tail", "ora_planck_head", "ora_coef_c4", "ora_coef_w", "ora_coef_c2_over_dt",
                  "ora_coef_c4_ds", "ora_coef_w_ds", "ora_coef_c2_over_dt_ds", "ora_coef_c5_over_dt",
                  "ora_coef_w5_over_dt"):
            getattr(L, f).argtypes = [_d]
            getattr(L, f).restype = _d
        for f in ("ora_phi_group", "ora_dphi_group"):
            getattr(L, f).argtypes = [_d, _d, _d, _d, _d]
            getattr(L, f).restype = _d
        L.ora_freq_slope.argtypes = [_d, _d, _d]
        L.ora_freq_slope.restype = _d
        L.ora_linear_offset.argtypes = [_d, _d]
        L.ora_linear_offset.restype = _d
        L.ora_sample_nu.argtypes = [_d, _d, _d, _d]
        L.ora_sample_nu.restype = _d
        L.ora_create.argtypes = [C.POINTER(Params)]
        L.ora_create.restype = C.c_void_p
        L.ora_destroy.argtypes = [C.c_void_p]
        L.ora_set_opacity.argtypes = [C.c_void_p, _pd]
        L.ora_set_material.argtypes = [C.c_void_p, _pd, _pd, _pd, _pu8]
        L.ora_step.argtypes = [C.c_void_p, C.c_int]
        L.ora_get_fields.argtypes = [C.c_void_p, _pd, _pd, _pd]
        L.ora_get_tallies.argtypes = [C.c_void_p, _pd, _pd, _pd, _pd, _pi64, _pd, _pd]
        L.ora_pool_size.argtypes = [C.c_void_p]
        L.ora_pool_size.restype = C.c_int64
        L.ora_get_pool.argtypes = [C.c_void_p, _pd, _pd, _pd, _pd, _pd, _pd, _pu64, _pi32, _pi32]
        L.ora_set_pool.argtypes = [C.c_void_p, C.c_int64, _pd, _pd, _pd, _pd, _pd, _pd, _pu64,
                                   _pi32, _pi32, C.c_uint64, _pd]
        L.ora_set_fields.argtypes = [C.c_void_p, _pd, _pd, C.c_int]
        L.ora_get_diag.argtypes = [C.c_void_p, C.POINTER(Diag)]
        L.ora_get_counters.argtypes = [C.c_void_p, _pu64, C.POINTER(C.c_int)]
        L.ora_get_start_weights.argtypes = [C.c_void_p, _pd]
        L.ora_record.argtypes = [C.c_void_p, C.c_int]
        L.ora_set_source.argtypes = [C.c_void_p, _pd, _d]
        L.ora_set_heat_capacity.argtypes = [C.c_void_p, _pd, _pd]
        L.ora_set_source_planck.argtypes = [C.c_void_p, _pd, _d, _d]
        L.ora_set_opacity_table.argtypes = [C.c_void_p, C.c_int, _pi32, C.c_int, _pd, C.c_int, _pd, _pd]
        L.ora_table_sigma.argtypes = [C.c_void_p, C.c_int, _d, _d]
        L.ora_table_sigma.restype = _d
        L.ora_olson_alpha.argtypes = [_d, _d, _pd]
        L.ora_olson_alpha.restype = _d
        L.ora_heat_capacity.argtypes = [C.c_void_p, C.c_int, _d]
        L.ora_heat_capacity.restype = _d
        L.ora_material_energy.argtypes = [C.c_void_p, C.c_int, _d]
        L.ora_material_energy.restype = _d
        L.ora_adjoint.argtypes = [C.c_void_p, _pd, _pd]
        L.ora_replay_frozen.argtypes = [C.c_void_p, _pd, _pd]
        L.ora_adjoint_updates.argtypes = []
        L.ora_adjoint_updates.restype = C.c_longlong
        _lib = L
    return _lib


def _p(a, t=_pd):
    return a.ctypes.data_as(t) if a is not None else None


# ---------------- scalar functions ----------------

def philox(ctr, key):
    c = (C.c_uint32 * 4)(*[int(v) & 0xFFFFFFFF for v in ctr])
    k = (C.c_uint32 * 2)(*[int(v) & 0xFFFFFFFF for v in key])
    o = (C.c_uint32 * 4)()
    lib().ora_philox4x32_10(c, k, o)
    return [int(v) for v in o]


def uniform(seed, pid, step, purpose, d):
    return lib().ora_uniform(seed, pid, step, purpose, d)


def olson_alpha(T, chi):
    d = C.c_double()
    a = lib().ora_olson_alpha(T, chi, C.byref(d))
    return a, d.value


def planck_tail(x):
    return lib().ora_planck_tail(x)


def planck_head(x):
    return lib().ora_planck_head(x)


def phi_group(T, nl, nh, a=1.0, c=1.0):
    return lib().ora_phi_group(T, nl, nh, a, c)


def dphi_group(T, nl, nh, a=1.0, c=1.0):
    return lib().ora_dphi_group(T, nl, nh, a, c)


def coef_c4(s):
    return lib().ora_coef_c4(s)


def coef_w(s):
    return lib().ora_coef_w(s)


def coef_c2_over_dt(s):
    return lib().ora_coef_c2_over_dt(s)


def coef_c5_over_dt(s):
    return lib().ora_coef_c5_over_dt(s)


def coef_w5_over_dt(s):
    return lib().ora_coef_w5_over_dt(s)


def linear_offset(beta, U):
    return lib().ora_linear_offset(beta, U)


def coef_c4_ds(s):
    return lib().ora_coef_c4_ds(s)


def coef_w_ds(s):
    return lib().ora_coef_w_ds(s)


def coef_c2_over_dt_ds(s):
    return lib().ora_coef_c2_over_dt_ds(s)


def freq_slope(nl, nh, T):
    return lib().ora_freq_slope(nl, nh, T)


def sample_nu(nl, nh, beta, U):
    return lib().ora_sample_nu(nl, nh, beta, U)


# ---------------- simulation ----------------

class OracleError(RuntimeError):
    def __init__(self, code, where):
        super().__init__(f"oracle {where} failed with status {code}")
        self.code = code


class Sim:
    """One problem instance advanced by the oracle."""

    def __init__(self, prob):
        L = lib()
        self.prob = prob
        self._nu = np.ascontiguousarray(prob.nu_edges, dtype=np.float64)
        P = Params()
        P.dim, P.nx, P.ny = prob.dim, prob.nx, prob.ny
        P.x0, P.x1, P.y0, P.y1 = prob.x0, prob.x1, prob.y0, prob.y1
        for k in range(4):
            P.bc[k] = int(prob.bc[k])
            P.bcT[k] = float(prob.bcT[k])
        P.G = prob.G
        P.nu = _p(self._nu)
        P.nu_power = prob.nu_power
        P.c, P.a, P.eps, P.dt, P.w_ref = prob.c, prob.a, prob.eps, prob.dt, prob.w_ref
        P.n_cap, P.seed, P.pool_cap = prob.n_cap, prob.seed, prob.pool_cap
        P.si_max_iters, P.si_tol, P.flags = prob.si_max_iters, prob.si_tol, prob.flags
        P.tau_num_C, P.tau_num_jump = prob.tau_num_C, prob.tau_num_jump
        P.T_power = prob.T_power
        P.opacity_stim = prob.opacity_stim
        self._P = P
        h = L.ora_create(C.byref(P))
        if not h:
            raise OracleError(EINVAL, "create")
        self.h = h
        kap = np.ascontiguousarray(prob.kappa, dtype=np.float64)
        st = L.ora_set_opacity(h, _p(kap))
        if st:
            raise OracleError(st, "set_opacity")
        if prob.opacity_table is not None:
            t = prob.opacity_table
            self._tab = (np.ascontiguousarray(t["mat"], dtype=np.int32), np.ascontiguousarray(t["nu"], dtype=np.float64),
                         np.ascontiguousarray(t["T"], dtype=np.float64), np.ascontiguousarray(t["sigma"], dtype=np.float64))
            m, nu, T, sg = self._tab
            st = L.ora_set_opacity_table(h, int(sg.shape[0]), _p(m, _pi32), len(nu), _p(nu), len(T), _p(T), _p(sg))
            if st:
                raise OracleError(st, "set_opacity_table")
        if prob.olson_H is not None:
            self._ol = (np.ascontiguousarray(prob.olson_H, dtype=np.float64),
                        np.ascontiguousarray(prob.olson_chi, dtype=np.float64))
            st = L.ora_set_heat_capacity(h, _p(self._ol[0]), _p(self._ol[1]))
            if st:
                raise OracleError(st, "set_heat_capacity")
        if prob.source_shape is not None:
            self._qf = np.ascontiguousarray(prob.source_shape, dtype=np.float64)
            st = L.ora_set_source_planck(h, _p(self._qf), float(prob.source_T), float(prob.source_t_off))
            if st:
                raise OracleError(st, "set_source_planck")
        if prob.source is not None:
            q = np.ascontiguousarray(prob.source, dtype=np.float64)
            st = L.ora_set_source(h, _p(q), float(prob.source_t_off))
            if st:
                raise OracleError(st, "set_source")
        cv = np.ascontiguousarray(prob.cv, dtype=np.float64)
        T0 = np.ascontiguousarray(prob.T0, dtype=np.float64)
        Tr0 = np.ascontiguousarray(prob.Tr0, dtype=np.float64)
        pin = np.ascontiguousarray(prob.pinned, dtype=np.uint8)
        st = L.ora_set_material(h, _p(cv), _p(T0), _p(Tr0), _p(pin, _pu8))
        if st:
            raise OracleError(st, "set_material")

    def close(self):
        if getattr(self, "h", None):
            lib().ora_destroy(self.h)
            self.h = None

    def __del__(self):
        self.close()

    def table_sigma(self, m, nu, T):
        return lib().ora_table_sigma(self.h, int(m), float(nu), float(T))

    def heat_capacity(self, cell, T):
        return lib().ora_heat_capacity(self.h, int(cell), float(T))

    def material_energy(self, cell, T):
        return lib().ora_material_energy(self.h, int(cell), float(T))

    def step(self, n=1, check=True):
        st = lib().ora_step(self.h, n)
        if check and st:
            raise OracleError(st, "step")
        return st

    def set_opacity(self, kappa):
        kap = np.ascontiguousarray(kappa, dtype=np.float64)
        st = lib().ora_set_opacity(self.h, _p(kap))
        if st:
            raise OracleError(st, "set_opacity")

    def fields(self):
        p = self.prob
        rho = np.zeros((p.ncell, p.G))
        T = np.zeros(p.ncell)
        rhop = np.zeros((p.ncell, p.G))
        lib().ora_get_fields(self.h, _p(rho), _p(T), _p(rhop))
        return rho, T, rhop

    def tallies(self):
        p = self.prob
        G = p.G
        fx = np.zeros(((p.nx + 1) * p.ny, G, 2))
        fy = np.zeros((p.nx * (p.ny + 1), G, 2))
        dep = np.zeros((p.ncell, G))
        surv = np.zeros((p.ncell, G))
        nb = np.zeros((p.ncell, G), np.int64)
        wnew = np.zeros((p.ncell, G))
        Q = np.zeros((p.ncell, G))
        lib().ora_get_tallies(self.h, _p(fx), _p(fy), _p(dep), _p(surv), _p(nb, _pi64), _p(wnew), _p(Q))
        return dict(fx=fx, fy=fy if p.dim == 2 else None, dep=dep, surv=surv, nbirth=nb, wnew=wnew, Q=Q)

    def start_weights(self):
        p = self.prob
        st = np.zeros((p.ncell, p.G))
        lib().ora_get_start_weights(self.h, _p(st))
        return st

    def pool(self):
        n = lib().ora_pool_size(self.h)
        out = dict(x=np.zeros(n), y=np.zeros(n), ox=np.zeros(n), oy=np.zeros(n), nu=np.zeros(n),
                   w=np.zeros(n), id=np.zeros(n, np.uint64), cell=np.zeros(n, np.int32),
                   g=np.zeros(n, np.int32))
        lib().ora_get_pool(self.h, _p(out["x"]), _p(out["y"]), _p(out["ox"]), _p(out["oy"]),
                           _p(out["nu"]), _p(out["w"]), _p(out["id"], _pu64),
                           _p(out["cell"], _pi32), _p(out["g"], _pi32))
        return out

    def set_pool(self, pool, birth_counter, rhop=None):
        n = len(pool["x"])
        arr = {k: np.ascontiguousarray(pool[k]) for k in pool}
        st = lib().ora_set_pool(self.h, n, _p(arr["x"]), _p(arr.get("y")), _p(arr["ox"]),
                                _p(arr.get("oy")), _p(arr["nu"]), _p(arr["w"]),
                                _p(arr["id"].astype(np.uint64), _pu64),
                                _p(arr["cell"].astype(np.int32), _pi32),
                                _p(arr["g"].astype(np.int32), _pi32), int(birth_counter),
                                _p(np.ascontiguousarray(rhop)) if rhop is not None else None)
        if st:
            raise OracleError(st, "set_pool")

    def set_fields(self, rho, T, step):
        st = lib().ora_set_fields(self.h, _p(np.ascontiguousarray(rho, dtype=np.float64)),
                                  _p(np.ascontiguousarray(T, dtype=np.float64)), int(step))
        if st:
            raise OracleError(st, "set_fields")

    def state(self):
        """The whole state a step starts from: fields, pool and counters."""
        rho, T, rhop = self.fields()
        births, step = self.counters()
        return dict(rho=rho, T=T, rhop=rhop, pool=self.pool(), births=births, step=step)

    def restore(self, st):
        self.set_fields(st["rho"], st["T"], st["step"])
        self.set_pool(st["pool"], st["births"], st["rhop"])

    def diag(self):
        d = Diag()
        lib().ora_get_diag(self.h, C.byref(d))
        return d.as_dict()

    def counters(self):
        b = C.c_uint64()
        s = C.c_int()
        lib().ora_get_counters(self.h, C.byref(b), C.byref(s))
        return int(b.value), int(s.value)

    def record(self, on=True):
        st = lib().ora_record(self.h, 1 if on else 0)
        if st:
            raise OracleError(st, "record")

    def adjoint(self, dJdT):
        p = self.prob
        g = np.zeros((p.ncell, p.G))
        d = np.ascontiguousarray(dJdT, dtype=np.float64)
        st = lib().ora_adjoint(self.h, _p(d), _p(g))
        if st:
            raise OracleError(st, "adjoint")
        return g

    def adjoint_updates(self):
        """(cell, group) updates of the transposed iterations of the last adjoint call."""
        return int(lib().ora_adjoint_updates())

    def replay_frozen(self, kappa):
        p = self.prob
        T = np.zeros(p.ncell)
        k = np.ascontiguousarray(kappa, dtype=np.float64)
        st = lib().ora_replay_frozen(self.h, _p(k), _p(T))
        if st:
            raise OracleError(st, "replay_frozen")
        return T
