"""ctypes wrapper of the FP64 CPU oracle (oracle/liborc.so).

TEST INFRASTRUCTURE ONLY: imported by tests/, by the smoke check and by the
CPU-baseline leg of bench.py.  The product library never uses it.
"""
import ctypes as C
import os

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_LIB_PATH = os.path.join(_HERE, "liborc.so")
_lib = None


class OrcCfg(C.Structure):
    _fields_ = [
        ("a", C.c_double), ("b", C.c_double), ("L", C.c_double),
        ("nr", C.c_int), ("nz", C.c_int),
        ("V_inner", C.c_double), ("V_outer", C.c_double), ("V_end", C.c_double),
        ("end_mode", C.c_int),
        ("B0", C.c_double), ("mirror_k", C.c_double),
        ("p_mbar", C.c_double), ("T_gas_K", C.c_double), ("M_gas_amu", C.c_double),
        ("sigma_el", C.c_double), ("iz_I_eV", C.c_double), ("lotz_a", C.c_double),
        ("lotz_q", C.c_double), ("opal_Ebar_eV", C.c_double), ("okh_xi", C.c_double),
        ("E_cap_eV", C.c_double),
        ("n_init", C.c_int64), ("r_lo", C.c_double), ("r_hi", C.c_double),
        ("z_lo", C.c_double), ("z_hi", C.c_double), ("T_init_eV", C.c_double),
        ("weight", C.c_double), ("load_mode", C.c_int),
        ("seed", C.c_uint64), ("dt", C.c_double),
        ("fx_shift", C.c_int), ("diag_interval", C.c_int), ("collisions", C.c_int),
        ("src_rate", C.c_double), ("src_T_eV", C.c_double),
        ("ins_r0", C.c_double), ("ins_z0", C.c_double), ("ins_er", C.c_double), ("ins_ez", C.c_double),
        ("ins_band", C.c_double), ("spline_order", C.c_int), ("okh_E0_eV", C.c_double),
    ]


class OrcDerived(C.Structure):
    _fields_ = [(n, C.c_double) for n in (
        "dr", "dz", "inv_dr", "inv_dz", "h", "n_n", "v_cap", "sig_iz_max", "nu_prime",
        "P_null", "nsig_el", "lotz_aq", "half_me_over_e", "two_e_over_me", "mass_ratio2",
        "two_S", "inv_two_S", "bscale")]


class OrcDiag(C.Structure):
    _fields_ = [
        ("step", C.c_int64), ("n_live", C.c_int64),
        ("n_elastic", C.c_int64), ("n_ioniz", C.c_int64), ("n_null_cand", C.c_int64),
        ("n_cap_overflow", C.c_int64),
        ("n_absorbed", C.c_int64 * 4), ("absorbed_W", C.c_int64 * 4),
        ("total_Q", C.c_int64), ("n_samples", C.c_int64),
        ("I_wall", C.c_double * 4), ("peak_density", C.c_double),
        ("peak_I_outer", C.c_double), ("peak_I_inner", C.c_double),
        ("n_source", C.c_int64),
        ("n_nonfinite", C.c_int64),
    ]


_D = C.POINTER(C.c_double)
_I64 = C.POINTER(C.c_int64)
_U64 = C.POINTER(C.c_uint64)
_U32 = C.POINTER(C.c_uint32)


def lib():
    global _lib
    if _lib is None:
        if not os.path.exists(_LIB_PATH):
            from . import build as _b
            _b.build()
        L = C.CDLL(_LIB_PATH)
        L.orc_philox4x32_10.argtypes = [_U32, _U32, _U32]
        L.orc_u52.argtypes = [C.c_uint32, C.c_uint32]
        L.orc_u52.restype = C.c_double
        L.orc_derive.argtypes = [C.POINTER(OrcCfg), C.POINTER(OrcDerived)]
        L.orc_auto_shift.argtypes = [C.c_double]
        L.orc_auto_shift.restype = C.c_int
        L.orc_okh_cos.argtypes = [C.c_double, C.c_double]
        L.orc_okh_cos.restype = C.c_double
        L.orc_opal_split.argtypes = [C.c_double, C.c_double, C.c_double]
        L.orc_opal_split.restype = C.c_double
        L.orc_scatter.argtypes = [C.c_double] * 5 + [_D]
        L.orc_sigma_iz.argtypes = [C.POINTER(OrcCfg), C.c_double]
        L.orc_sigma_iz.restype = C.c_double
        L.orc_bfield.argtypes = [C.POINTER(OrcCfg), _D, _D]
        L.orc_vacuum.argtypes = [C.POINTER(OrcCfg), _D]
        L.orc_solve.argtypes = [C.POINTER(OrcCfg), _D, _D]
        L.orc_poisson_charge.argtypes = [C.POINTER(OrcCfg), _I64, _D]
        L.orc_efield.argtypes = [C.POINTER(OrcCfg), _D, _D, _D]
        L.orc_node_volume.argtypes = [C.POINTER(OrcCfg), _D]
        L.orc_deposit_one.argtypes = [C.POINTER(OrcCfg), C.c_double, C.c_double, C.c_double, _I64]
        L.orc_xs_bound.argtypes = [C.c_double]
        L.orc_xs_bound.restype = C.c_double
        L.orc_null_candidates.argtypes = [C.POINTER(OrcCfg), C.c_uint32, C.c_int64, _U64, C.POINTER(C.c_uint8)]
        L.orc_xi_sc.argtypes = [C.c_double, C.c_double]
        L.orc_xi_sc.restype = C.c_double
        L.orc_deposit_f32.argtypes = [C.POINTER(OrcCfg), C.c_int64, _D, _D, _D, _I64]
        L.orc_create.argtypes = [C.POINTER(OrcCfg), C.c_int64]
        L.orc_create.restype = C.c_void_p
        L.orc_destroy.argtypes = [C.c_void_p]
        L.orc_load.argtypes = [C.c_void_p]
        L.orc_set_particles.argtypes = [C.c_void_p, C.c_int64] + [_D] * 6 + [_U64]
        L.orc_get_particles.argtypes = [C.c_void_p, C.c_int64] + [_D] * 6 + [_U64]
        L.orc_get_particles.restype = C.c_int64
        L.orc_set_fields.argtypes = [C.c_void_p, _D, _D, _D, _D, C.c_int]
        L.orc_get_fields.argtypes = [C.c_void_p, _D, _D, _D, _D]
        L.orc_set_step.argtypes = [C.c_void_p, C.c_int64]
        L.orc_step.argtypes = [C.c_void_p, C.c_int]
        L.orc_get_charge.argtypes = [C.c_void_p, _I64]
        L.orc_get_charge_w.argtypes = [C.c_void_p, _I64]
        L.orc_get_phi.argtypes = [C.c_void_p, _D]
        L.orc_get_diag.argtypes = [C.c_void_p, C.POINTER(OrcDiag)]
        L.orc_get_time_avg_density.argtypes = [C.c_void_p, _D]
        L.orc_moments.argtypes = [C.c_void_p, _D]
        L.orc_well_depth.argtypes = [C.POINTER(OrcCfg), _D, C.c_int, _D, _D, _D]
        L.orc_num_threads.restype = C.c_int
        L.orc_load.restype = C.c_int
        L.orc_set_cross_sections.argtypes = [C.c_void_p, C.c_int, _D, _D, _D]
        L.orc_set_cross_sections.restype = C.c_int
        L.orc_set_anisotropy.argtypes = [C.c_void_p, C.c_int, _D, _D]
        L.orc_set_anisotropy.restype = C.c_int
        L.orc_get_charge3.argtypes = [C.c_void_p, _I64]
        L.orc_get_coef3.argtypes = [C.c_void_p, _D]
        L.orc_s3_weights.argtypes = [C.c_double, _D, _D]
        L.orc_s3_poisson_fn.argtypes = [C.POINTER(OrcCfg), _FN, C.c_void_p, _D]
        L.orc_is3_poisson_fn.argtypes = [C.POINTER(OrcCfg), _FN, C.c_void_p, _D]
        L.orc_is3_poisson_fn.restype = C.c_int
        L.orc_is3_phi_at.argtypes = [C.POINTER(OrcCfg), _D, C.c_double, C.c_double]
        L.orc_is3_phi_at.restype = C.c_double
        L.orc_is3_field.argtypes = [C.POINTER(OrcCfg), _D, C.c_double, C.c_double, _D, _D]
        L.orc_is3_info.argtypes = [C.POINTER(OrcCfg), C.POINTER(C.c_int), C.POINTER(C.c_int), C.POINTER(C.c_int)]
        L.orc_is3_info.restype = C.c_int
        L.orc_get_charge3w.argtypes = [C.c_void_p, _I64]
        L.orc_s3_poisson_fn.restype = C.c_int
        L.orc_s3_phi_at.argtypes = [C.POINTER(OrcCfg), _D, C.c_double, C.c_double]
        L.orc_s3_phi_at.restype = C.c_double
        L.orc_s3_field.argtypes = [C.POINTER(OrcCfg), _D, C.c_double, C.c_double, _D, _D]
        L.orc_s3_deposit.argtypes = [C.POINTER(OrcCfg), C.c_double, C.c_double, C.c_int64, _I64]
        L.orc_sim_derived.argtypes = [C.c_void_p, C.POINTER(OrcDerived)]
        L.orc_xs_at.argtypes = [C.c_int, _D, _D, C.c_double]
        L.orc_xs_at.restype = C.c_double
        L.orc_xs_sigv_max.argtypes = [C.POINTER(OrcCfg), C.c_int, _D, _D, _D]
        L.orc_xs_sigv_max.restype = C.c_double
        L.orc_ins_g.argtypes = [C.POINTER(OrcCfg), C.c_double, C.c_double]
        L.orc_ins_g.restype = C.c_double
        L.orc_ins_gamma.argtypes = [C.POINTER(OrcCfg)]
        L.orc_ins_gamma.restype = C.c_double
        L.orc_ins_wp.argtypes = [C.POINTER(OrcCfg), C.c_double, C.c_double]
        L.orc_ins_wp.restype = C.c_double
        L.orc_ins_weight.argtypes = [C.POINTER(OrcCfg), C.c_double, C.c_double, _D, _D]
        L.orc_ins_weight.restype = C.c_double
        L.orc_ins_check.argtypes = [C.POINTER(OrcCfg)]
        L.orc_ins_check.restype = C.c_int
        L.orc_ins_classify.argtypes = [C.POINTER(OrcCfg), C.POINTER(C.c_int)]
        L.orc_ins_classify.restype = C.c_int
        L.orc_ins_info.argtypes = [C.POINTER(OrcCfg), C.POINTER(C.c_int), C.POINTER(C.c_int), C.POINTER(C.c_int)]
        L.orc_ins_info.restype = C.c_int
        L.orc_ins_poisson_fn.argtypes = [C.POINTER(OrcCfg), _FN, C.c_void_p, _D]
        L.orc_ins_poisson_fn.restype = C.c_int
        _lib = L
    return _lib


_FN = C.CFUNCTYPE(C.c_double, C.c_double, C.c_double, C.c_void_p)


def _dp(a):
    return a.ctypes.data_as(_D)


def make_cfg(d, fx_shift=None):
    c = OrcCfg()
    for name, _ in OrcCfg._fields_:
        if name in d:
            setattr(c, name, d[name])
    if fx_shift is not None:
        c.fx_shift = int(fx_shift)
    elif c.fx_shift == 0:
        c.fx_shift = auto_shift(d["weight"])
    return c


# ---- unit functions -------------------------------------------------------

def philox(ctr, key):
    ctr = (C.c_uint32 * 4)(*[int(x) & 0xFFFFFFFF for x in ctr])
    key = (C.c_uint32 * 2)(*[int(x) & 0xFFFFFFFF for x in key])
    out = (C.c_uint32 * 4)()
    lib().orc_philox4x32_10(ctr, key, out)
    return list(out)


def u52(hi, lo):
    return lib().orc_u52(hi, lo)


def derive(d, fx_shift=None):
    c = make_cfg(d, fx_shift)
    out = OrcDerived()
    lib().orc_derive(C.byref(c), C.byref(out))
    return {n: getattr(out, n) for n, _ in OrcDerived._fields_}


def auto_shift(w_max):
    return lib().orc_auto_shift(float(w_max))


def okh_cos(xi, u):
    return lib().orc_okh_cos(xi, u)


def opal_split(Ebar, E_av, u):
    return lib().orc_opal_split(Ebar, E_av, u)


def scatter(u, cosx, phi):
    out = (C.c_double * 3)()
    lib().orc_scatter(float(u[0]), float(u[1]), float(u[2]), float(cosx), float(phi), out)
    return np.array(list(out))


def sigma_iz(d, E):
    c = make_cfg(d)
    return lib().orc_sigma_iz(C.byref(c), float(E))


def _nodes(d):
    return (d["nr"] + 1) * (d["nz"] + 1)


def _shape(d):
    return (d["nr"] + 1, d["nz"] + 1)


def bfield(d):
    c = make_cfg(d)
    Br = np.zeros(_nodes(d)); Bz = np.zeros(_nodes(d))
    lib().orc_bfield(C.byref(c), _dp(Br), _dp(Bz))
    return Br.reshape(_shape(d)), Bz.reshape(_shape(d))


def vacuum(d):
    c = make_cfg(d)
    phi = np.zeros(_nodes(d))
    lib().orc_vacuum(C.byref(c), _dp(phi))
    return phi.reshape(_shape(d))


def solve(d, rhs):
    c = make_cfg(d)
    rhs = np.ascontiguousarray(rhs, dtype=np.float64).reshape(-1)
    phi = np.zeros(_nodes(d))
    lib().orc_solve(C.byref(c), _dp(rhs), _dp(phi))
    return phi.reshape(_shape(d))


def poisson_charge(d, Q, fx_shift=None):
    c = make_cfg(d, fx_shift)
    Q = np.ascontiguousarray(Q, dtype=np.int64).reshape(-1)
    phi = np.zeros(_nodes(d))
    lib().orc_poisson_charge(C.byref(c), Q.ctypes.data_as(_I64), _dp(phi))
    return phi.reshape(_shape(d))


def efield(d, phi):
    c = make_cfg(d)
    phi = np.ascontiguousarray(phi, dtype=np.float64).reshape(-1)
    Er = np.zeros(_nodes(d)); Ez = np.zeros(_nodes(d))
    lib().orc_efield(C.byref(c), _dp(phi), _dp(Er), _dp(Ez))
    return Er.reshape(_shape(d)), Ez.reshape(_shape(d))


def node_volume(d):
    c = make_cfg(d)
    V = np.zeros(_nodes(d))
    lib().orc_node_volume(C.byref(c), _dp(V))
    return V.reshape(_shape(d))


def deposit_one(d, r, z, w, fx_shift=None):
    c = make_cfg(d, fx_shift)
    Q = np.zeros(_nodes(d), dtype=np.int64)
    lib().orc_deposit_one(C.byref(c), float(r), float(z), float(w), Q.ctypes.data_as(_I64))
    return Q.reshape(_shape(d))


def deposit_f32(d, r, z, w, fx_shift=None):
    """The deposit of particles (r, z, w) taken in single precision from their
    FP32 values: the node charges the batched FP32 form must produce."""
    c = make_cfg(d, fx_shift)
    r, z, w = (np.ascontiguousarray(a, dtype=np.float64) for a in (r, z, w))
    Q = np.zeros(_nodes(d), dtype=np.int64)
    lib().orc_deposit_f32(C.byref(c), len(r), _dp(r), _dp(z), _dp(w), Q.ctypes.data_as(_I64))
    return Q.reshape(_shape(d))


def null_candidates(d, step, keys):
    """Boolean mask: which electrons (by key) are null-collision candidates
    at `step` (the analytic model's P_null)."""
    c = make_cfg(d)
    keys = np.ascontiguousarray(keys, dtype=np.uint64)
    out = np.zeros(len(keys), dtype=np.uint8)
    lib().orc_null_candidates(C.byref(c), int(step) & 0xFFFFFFFF, len(keys), keys.ctypes.data_as(_U64),
                              out.ctypes.data_as(C.POINTER(C.c_uint8)))
    return out.astype(bool)


def well_depth(d, phi, r_mid):
    """Well depth (V) and the position of the potential maximum along the
    field lines through r_mid at the midplane."""
    c = make_cfg(d)
    phi = np.ascontiguousarray(phi, dtype=np.float64).reshape(-1)
    r = np.ascontiguousarray(r_mid, dtype=np.float64)
    dep = np.zeros(len(r))
    zm = np.zeros(len(r))
    lib().orc_well_depth(C.byref(c), _dp(phi), len(r), _dp(r), _dp(dep), _dp(zm))
    return dep, zm


# ---- elliptic insert ------------------------------------------------------

def ins_g(d, r, z):
    return lib().orc_ins_g(C.byref(make_cfg(d)), float(r), float(z))


def ins_gamma(d):
    return lib().orc_ins_gamma(C.byref(make_cfg(d)))


def ins_weight(d, r, z):
    """Weight function value and gradient (w, dw/dr, dw/dz)."""
    wr = np.zeros(1); wz = np.zeros(1)
    w = lib().orc_ins_weight(C.byref(make_cfg(d)), float(r), float(z), _dp(wr), _dp(wz))
    return w, float(wr[0]), float(wz[0])


def ins_classify(d):
    """Node classes: 0 not an unknown, 1 inner, 2 outer, 3 exterior."""
    cls = np.zeros(_nodes(d), dtype=np.int32)
    if lib().orc_ins_classify(C.byref(make_cfg(d)), cls.ctypes.data_as(C.POINTER(C.c_int))) != 0:
        raise ValueError("insert configuration refused")
    return cls.reshape(_shape(d))


def ins_info(d):
    n = C.c_int(); bw = C.c_int(); cnt = (C.c_int * 4)()
    if lib().orc_ins_info(C.byref(make_cfg(d)), C.byref(n), C.byref(bw), cnt) != 0:
        raise ValueError("insert configuration refused")
    return {"unknowns": n.value, "bandwidth": bw.value, "counts": list(cnt)}


def ins_poisson_fn(d, f):
    """Nodal web-spline solution of -lap(phi) = f(r, z) with phi = 0 on every
    electrode (the manufactured-solution hook)."""
    cb = _FN(lambda r, z, u: float(f(r, z)))
    phi = np.zeros(_nodes(d))
    if lib().orc_ins_poisson_fn(C.byref(make_cfg(d)), cb, None, _dp(phi)) != 0:
        raise ValueError("insert configuration refused")
    return phi.reshape(_shape(d))


def xs_at(E, s, x):
    E = np.ascontiguousarray(E, dtype=np.float64)
    s = np.ascontiguousarray(s, dtype=np.float64)
    return lib().orc_xs_at(len(E), _dp(E), _dp(s), float(x))


def xi_sc(E0, E):
    return lib().orc_xi_sc(float(E0), float(E))


def xs_bound(sigv_max):
    return lib().orc_xs_bound(float(sigv_max))


def xs_sigv_max(d, E, el, iz):
    a = [np.ascontiguousarray(x, dtype=np.float64) for x in (E, el, iz)]
    return lib().orc_xs_sigv_max(C.byref(make_cfg(d)), len(a[0]), *[_dp(x) for x in a])


# ---- cubic B-spline shapes --------------------------------------------------

def _ext(d):
    return (d["nr"] + 3) * (d["nz"] + 3)


def s3_weights(f):
    w = np.zeros(4); dw = np.zeros(4)
    lib().orc_s3_weights(float(f), _dp(w), _dp(dw))
    return w, dw


def s3_deposit(d, r, z, Wq):
    """Ghosted ((nr+3) x (nz+3)) cubic deposit of one particle of Wq units."""
    Qx = np.zeros(_ext(d), dtype=np.int64)
    lib().orc_s3_deposit(C.byref(make_cfg(d)), float(r), float(z), int(Wq), Qx.ctypes.data_as(_I64))
    return Qx.reshape(d["nr"] + 3, d["nz"] + 3)


def s3_poisson_fn(d, f):
    """Ghosted cubic coefficients of the solution of -lap(phi) = f with phi = 0
    on the four walls (manufactured-solution hook)."""
    cb = _FN(lambda r, z, u: float(f(r, z)))
    cx = np.zeros(_ext(d))
    if lib().orc_s3_poisson_fn(C.byref(make_cfg(d)), cb, None, _dp(cx)) != 0:
        raise ValueError("cubic configuration refused")
    return cx


def s3_phi_at(d, cx, r, z):
    cx = np.ascontiguousarray(cx, dtype=np.float64).reshape(-1)
    return lib().orc_s3_phi_at(C.byref(make_cfg(d)), _dp(cx), float(r), float(z))


def s3_field(d, cx, r, z):
    cx = np.ascontiguousarray(cx, dtype=np.float64).reshape(-1)
    a = np.zeros(1); b = np.zeros(1)
    lib().orc_s3_field(C.byref(make_cfg(d)), _dp(cx), float(r), float(z), _dp(a), _dp(b))
    return float(a[0]), float(b[0])


def is3_poisson_fn(d, f):
    """Cubic web-splines with the insert: ghosted expanded coefficients of the
    solution of -lap(phi) = f, phi = 0 on the electrodes and the insert (zero
    z-derivative at open ends)."""
    cb = _FN(lambda r, z, u: float(f(r, z)))
    cx = np.zeros(_ext(d))
    if lib().orc_is3_poisson_fn(C.byref(make_cfg(d)), cb, None, _dp(cx)) != 0:
        raise ValueError("cubic insert configuration refused")
    return cx


def is3_phi_at(d, cx, r, z):
    cx = np.ascontiguousarray(cx, dtype=np.float64).reshape(-1)
    return lib().orc_is3_phi_at(C.byref(make_cfg(d)), _dp(cx), float(r), float(z))


def is3_field(d, cx, r, z):
    cx = np.ascontiguousarray(cx, dtype=np.float64).reshape(-1)
    a = np.zeros(1); b = np.zeros(1)
    lib().orc_is3_field(C.byref(make_cfg(d)), _dp(cx), float(r), float(z), _dp(a), _dp(b))
    return float(a[0]), float(b[0])


def is3_info(d):
    n, bw = C.c_int(), C.c_int()
    cnt = (C.c_int * 4)()
    if lib().orc_is3_info(C.byref(make_cfg(d)), C.byref(n), C.byref(bw), cnt) != 0:
        raise ValueError("cubic insert configuration refused")
    return dict(n_inner=n.value, bandwidth=bw.value, counts=list(cnt))


def num_threads():
    return lib().orc_num_threads()


# ---- simulation object ----------------------------------------------------

class Sim:
    """One oracle instance.  Mirrors the product library's calls."""

    def __init__(self, d, fx_shift=None, capacity=0):
        self.d = dict(d)
        self.cfg = make_cfg(d, fx_shift)
        self.S = self.cfg.fx_shift
        self.nodes = _nodes(d)
        self.shape = _shape(d)
        self.h = lib().orc_create(C.byref(self.cfg), int(capacity or d.get("n_init", 1024)))
        if not self.h:
            raise ValueError("oracle refused the configuration")

    def close(self):
        if self.h:
            lib().orc_destroy(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def load(self):
        if lib().orc_load(self.h) != 0:
            raise ValueError("load box intersects the insert")

    def set_particles(self, st):
        n = len(st["r"])
        arrs = [np.ascontiguousarray(st[k], dtype=np.float64) for k in ("r", "z", "vr", "vt", "vz", "w")]
        key = np.ascontiguousarray(st["key"], dtype=np.uint64)
        lib().orc_set_particles(self.h, n, *[_dp(a) for a in arrs], key.ctypes.data_as(_U64))

    def get_particles(self):
        n = self.diag()["n_live"]
        arrs = [np.zeros(n) for _ in range(6)]
        key = np.zeros(n, dtype=np.uint64)
        lib().orc_get_particles(self.h, n, *[_dp(a) for a in arrs], key.ctypes.data_as(_U64))
        return dict(zip(("r", "z", "vr", "vt", "vz", "w"), arrs), key=key)

    def set_fields(self, Er=None, Ez=None, Br=None, Bz=None, frozen=1):
        def p(a):
            if a is None:
                return None
            a = np.ascontiguousarray(a, dtype=np.float64).reshape(-1)
            self._keep.append(a)
            return _dp(a)
        self._keep = []
        lib().orc_set_fields(self.h, p(Er), p(Ez), p(Br), p(Bz), int(frozen))

    def get_fields(self):
        a = [np.zeros(self.nodes) for _ in range(4)]
        lib().orc_get_fields(self.h, *[_dp(x) for x in a])
        return {k: v.reshape(self.shape) for k, v in zip(("Er", "Ez", "Br", "Bz"), a)}

    def set_cross_sections(self, E=None, sigma_el=None, sigma_iz=None):
        """Tabulated cross sections (m^2) at increasing energies (eV); None
        returns to the constant elastic and Lotz ionisation model."""
        if E is None:
            st = lib().orc_set_cross_sections(self.h, 0, None, None, None)
        else:
            self._xs = [np.ascontiguousarray(a, dtype=np.float64) for a in (E, sigma_el, sigma_iz)]
            st = lib().orc_set_cross_sections(self.h, len(self._xs[0]), *[_dp(a) for a in self._xs])
        if st != 0:
            raise ValueError("cross-section table refused")

    def set_anisotropy(self, E=None, xi=None):
        """Tabulated anisotropy xi(E) of the scattering law at increasing
        energies (eV); None returns to the constant okh_xi."""
        if E is None:
            st = lib().orc_set_anisotropy(self.h, 0, None, None)
        else:
            self._xi = [np.ascontiguousarray(a, dtype=np.float64) for a in (E, xi)]
            st = lib().orc_set_anisotropy(self.h, len(self._xi[0]), *[_dp(a) for a in self._xi])
        if st != 0:
            raise ValueError("anisotropy table refused")

    def derived(self):
        out = OrcDerived()
        lib().orc_sim_derived(self.h, C.byref(out))
        return {n: getattr(out, n) for n, _ in OrcDerived._fields_}

    def set_step(self, step):
        lib().orc_set_step(self.h, int(step))

    def step(self, n=1):
        lib().orc_step(self.h, int(n))

    def charge(self):
        Q = np.zeros(self.nodes, dtype=np.int64)
        lib().orc_get_charge(self.h, Q.ctypes.data_as(_I64))
        return Q.reshape(self.shape)

    def charge3(self):
        Q = np.zeros(_ext(self.d), dtype=np.int64)
        lib().orc_get_charge3(self.h, Q.ctypes.data_as(_I64))
        return Q.reshape(self.d["nr"] + 3, self.d["nz"] + 3)

    def coef3(self):
        c = np.zeros(_ext(self.d))
        lib().orc_get_coef3(self.h, _dp(c))
        return c.reshape(self.d["nr"] + 3, self.d["nz"] + 3)

    def charge3w(self):
        Q = np.zeros(_ext(self.d), dtype=np.int64)
        lib().orc_get_charge3w(self.h, Q.ctypes.data_as(_I64))
        return Q.reshape(self.d["nr"] + 3, self.d["nz"] + 3)

    def band_charge(self):
        Q = np.zeros(self.nodes, dtype=np.int64)
        lib().orc_get_charge_w(self.h, Q.ctypes.data_as(_I64))
        return Q.reshape(self.shape)

    def phi(self):
        p = np.zeros(self.nodes)
        lib().orc_get_phi(self.h, _dp(p))
        return p.reshape(self.shape)

    def diag(self):
        dg = OrcDiag()
        lib().orc_get_diag(self.h, C.byref(dg))
        out = {}
        for name, _ in OrcDiag._fields_:
            v = getattr(dg, name)
            out[name] = list(v) if hasattr(v, "__len__") else v
        return out

    def moments(self):
        """ORC_NMOM (11) node arrays: n, n u_r, n u_t, n u_z, the six
        second moments (rr, rt, rz, tt, tz, zz) and sum w nu_m / V."""
        out = np.zeros(11 * self.nodes)
        lib().orc_moments(self.h, _dp(out))
        return out.reshape((11,) + self.shape)

    def time_avg_density(self):
        n = np.zeros(self.nodes)
        lib().orc_get_time_avg_density(self.h, _dp(n))
        return n.reshape(self.shape)
