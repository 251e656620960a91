"""Thin ctypes binding of libpicmcc.so (the C ABI in include/pic.h).

Functions carry the C names and only marshal arguments; every step of the
particle loop runs in the library's HIP kernels.  PyTorch provides the device
memory (its caching allocator, through the library's allocator callback) and
the stream.  There is no fallback: if the library is missing, loading fails.
"""
import ctypes as C
import os

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libpicmcc.so")

PIC_OK, PIC_EINVAL, PIC_ENOMEM, PIC_EDEVICE, PIC_ECAPACITY, PIC_EOVERFLOW, PIC_ESTATE = 0, -1, -2, -3, -4, -5, -6
PIC_ENONFINITE = -7
PIC_MODE_FP64_PLAIN, PIC_MODE_FP32_BATCHED = 0, 1
_STATUS = {0: "PIC_OK", -1: "PIC_EINVAL", -2: "PIC_ENOMEM", -3: "PIC_EDEVICE",
           -4: "PIC_ECAPACITY", -5: "PIC_EOVERFLOW", -6: "PIC_ESTATE", -7: "PIC_ENONFINITE"}


class PicError(RuntimeError):
    def __init__(self, status, msg):
        super().__init__(f"{_STATUS.get(status, status)}: {msg}")
        self.status = status


_ALLOC_FN = C.CFUNCTYPE(C.c_void_p, C.c_size_t, C.c_void_p)
_FREE_FN = C.CFUNCTYPE(None, C.c_void_p, C.c_void_p)


class pic_allocator(C.Structure):
    _fields_ = [("alloc", _ALLOC_FN), ("free", _FREE_FN), ("user", C.c_void_p)]


class pic_instance_cfg(C.Structure):
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
        ("n_init", C.c_longlong), ("r_lo", C.c_double), ("r_hi", C.c_double),
        ("z_lo", C.c_double), ("z_hi", C.c_double), ("T_init_eV", C.c_double),
        ("weight", C.c_double), ("load_mode", C.c_int),
        ("seed", C.c_ulonglong), ("dt", C.c_double),
        ("fx_shift", C.c_int), ("diag_interval", C.c_int), ("collisions", C.c_int),
        ("src_rate", C.c_double), ("src_T_eV", C.c_double),
        ("ins_r0", C.c_double), ("ins_z0", C.c_double), ("ins_er", C.c_double), ("ins_ez", C.c_double),
        ("ins_band", C.c_double), ("spline_order", C.c_int), ("okh_E0_eV", C.c_double),
    ]


class pic_run_cfg(C.Structure):
    _fields_ = [
        ("mode", C.c_int), ("n_instances", C.c_int), ("tile_r", C.c_int), ("tile_z", C.c_int),
        ("halo", C.c_int), ("sort_interval", C.c_int), ("chunk", C.c_int), ("use_graph", C.c_int),
        ("device", C.c_int), ("stream", C.c_void_p), ("alloc", pic_allocator),
        ("capacity_factor", C.c_double), ("capacity_min", C.c_longlong), ("lanes", C.c_int),
    ]


class pic_diag_t(C.Structure):
    _fields_ = [
        ("step", C.c_longlong), ("n_live", C.c_longlong), ("n_elastic", C.c_longlong),
        ("n_ioniz", C.c_longlong), ("n_null_cand", C.c_longlong), ("n_cap_overflow", C.c_longlong),
        ("n_spawn_dropped", C.c_longlong), ("n_absorbed", C.c_longlong * 4),
        ("absorbed_W", C.c_longlong * 4), ("total_Q", C.c_longlong), ("n_samples", C.c_longlong),
        ("S", C.c_int), ("total_charge_C", C.c_double), ("I_wall", C.c_double * 4),
        ("peak_density", C.c_double), ("peak_time_avg_density", C.c_double),
        ("peak_I_outer", C.c_double), ("peak_I_inner", C.c_double),
        ("particle_steps", C.c_longlong),
        ("n_far_deposit", C.c_longlong),
        ("n_source", C.c_longlong),
        ("n_nonfinite", C.c_longlong),
    ]


class pic_derived_t(C.Structure):
    _fields_ = [(n, C.c_double) for n in (
        "dr", "dz", "inv_dr", "inv_dz", "h", "n_n", "v_cap", "sig_iz_max", "nu_prime", "P_null",
        "nsig_el", "lotz_aq", "half_me_over_e", "two_e_over_me", "mass_ratio2", "two_S",
        "inv_two_S", "bscale")]


EXPORTS = ("pic_init", "pic_step", "pic_diag", "pic_destroy", "pic_last_error", "pic_sync",
           "pic_get_particles", "pic_set_particles", "pic_set_fields", "pic_get_fields",
           "pic_get_charge", "pic_get_phi", "pic_set_step", "pic_derive", "pic_auto_shift",
           "pic_timing", "pic_tuning", "pic_retune", "pic_autotune", "pic_reserve", "pic_capacity",
           "pic_moments", "pic_moments_noalloc", "pic_well_depth", "pic_get_band_charge", "pic_insert_layout",
           "pic_set_cross_sections", "pic_get_spline3", "pic_set_anisotropy")

_lib = None
_D = C.POINTER(C.c_double)
_LL = C.POINTER(C.c_longlong)
_ULL = C.POINTER(C.c_ulonglong)
_I = C.POINTER(C.c_int)


def lib():
    """Load libpicmcc.so (raises if it has not been built)."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH):
        raise RuntimeError(f"{LIB_PATH} is missing: build it with __graft_entry__.build()")
    # torch ships its own HIP runtime (same soname as the system one).  Load it
    # first so the library binds to that runtime: streams and device pointers
    # handed over by torch are only valid in the runtime that made them.
    try:
        import torch  # noqa: F401
    except ImportError:
        pass
    L = C.CDLL(LIB_PATH)
    vp = C.c_void_p
    L.pic_init.argtypes = [C.POINTER(pic_run_cfg), C.POINTER(pic_instance_cfg), C.POINTER(vp)]
    L.pic_step.argtypes = [vp, C.c_int]
    L.pic_diag.argtypes = [vp, C.c_int, C.POINTER(pic_diag_t), _D, _D]
    L.pic_destroy.argtypes = [vp]
    L.pic_last_error.argtypes = [vp]
    L.pic_last_error.restype = C.c_char_p
    L.pic_sync.argtypes = [vp]
    L.pic_get_particles.argtypes = [vp, C.c_int] + [_D] * 6 + [_ULL, C.c_longlong, _LL]
    L.pic_set_particles.argtypes = [vp, C.c_int, C.c_longlong] + [_D] * 6 + [_ULL]
    L.pic_set_fields.argtypes = [vp, C.c_int, _D, _D, _D, _D, C.c_int]
    L.pic_get_fields.argtypes = [vp, C.c_int, _D, _D, _D, _D]
    L.pic_get_charge.argtypes = [vp, C.c_int, _LL]
    L.pic_get_phi.argtypes = [vp, C.c_int, _D]
    L.pic_set_step.argtypes = [vp, C.c_longlong]
    L.pic_derive.argtypes = [C.POINTER(pic_instance_cfg), C.c_int, C.POINTER(pic_derived_t)]
    L.pic_auto_shift.argtypes = [C.c_double]
    L.pic_auto_shift.restype = C.c_int
    L.pic_timing.argtypes = [vp, C.c_int, _LL, _D]
    L.pic_tuning.argtypes = [vp, _I, _I, _I, _I, _I, _I, _I]
    L.pic_retune.argtypes = [vp, C.c_int, C.c_int, C.c_int, C.c_int]
    L.pic_autotune.argtypes = [vp, C.c_int, C.c_char_p, _I, _I, _I, _I, _D, _I]
    L.pic_reserve.argtypes = [vp, C.c_int, C.c_longlong]
    L.pic_capacity.argtypes = [vp, C.c_int, _LL, _LL]
    L.pic_moments.argtypes = [vp, C.c_int, _D]
    L.pic_moments_noalloc.argtypes = [vp, C.c_int, vp]
    L.pic_well_depth.argtypes = [vp, C.c_int, C.c_int, _D, _D, _D]
    L.pic_get_band_charge.argtypes = [vp, C.c_int, _LL]
    L.pic_insert_layout.argtypes = [C.POINTER(pic_instance_cfg), _I, _I, _LL]
    L.pic_set_cross_sections.argtypes = [vp, C.c_int, C.c_int, _D, _D, _D]
    L.pic_get_spline3.argtypes = [vp, C.c_int, _LL, _D]
    L.pic_set_anisotropy.argtypes = [vp, C.c_int, C.c_int, _D, _D]
    for name in EXPORTS:
        if name not in ("pic_last_error", "pic_auto_shift"):
            getattr(L, name).restype = C.c_int
    _lib = L
    return L


def _check(st, ctx=None):
    if st != PIC_OK:
        msg = lib().pic_last_error(ctx)
        raise PicError(st, msg.decode() if msg else "")
    return st


def make_instance_cfg(d):
    c = pic_instance_cfg()
    for name, _ in pic_instance_cfg._fields_:
        if name in d:
            setattr(c, name, d[name])
    return c


# ---- host-only calls -------------------------------------------------------

def pic_auto_shift(w_max):
    return lib().pic_auto_shift(float(w_max))


def pic_insert_layout(inst):
    """Host-only set-up of an instance's elliptic insert: node counts by
    class (not an unknown, inner, outer, inside the metal), the size m of the
    corrected node set and the entries of the correction."""
    c = make_instance_cfg(inst)
    counts = (C.c_int * 4)()
    m = C.c_int()
    nnz = C.c_longlong()
    _check(lib().pic_insert_layout(C.byref(c), counts, C.byref(m), C.byref(nnz)))
    return {"counts": list(counts), "m": m.value, "entries": nnz.value}


def pic_derive(inst, S=0):
    c = make_instance_cfg(inst)
    out = pic_derived_t()
    _check(lib().pic_derive(C.byref(c), int(S), C.byref(out)))
    return {n: getattr(out, n) for n, _ in pic_derived_t._fields_}


# ---- torch plumbing ----------------------------------------------------------

class _TorchAllocator:
    """Allocator callbacks backed by torch's caching allocator."""

    def __init__(self, device, stream):
        import torch
        self.torch = torch
        self.device = device
        self.stream = stream
        self.live = {}

        def _alloc(nbytes, user):
            try:
                p = torch.cuda.caching_allocator_alloc(int(nbytes), device=self.device, stream=self.stream)
            except Exception:
                return None
            self.live[p] = nbytes
            return p

        def _free(ptr, user):
            if ptr in self.live:
                del self.live[ptr]
                torch.cuda.caching_allocator_delete(ptr)

        self._a = _ALLOC_FN(_alloc)
        self._f = _FREE_FN(_free)

    def struct(self):
        return pic_allocator(self._a, self._f, None)


# ---- the C calls, marshalled -----------------------------------------------

def pic_init(instances, mode=PIC_MODE_FP64_PLAIN, device=0, stream=None, use_torch=True,
             tile_r=0, tile_z=0, halo=0, sort_interval=0, chunk=0, use_graph=2,
             capacity_factor=0.0, capacity_min=0, lanes=0):
    """Create a context for a list of instance dicts.  Returns (ctx, keep)
    where keep holds the callbacks that must outlive the context."""
    n = len(instances)
    arr = (pic_instance_cfg * n)(*[make_instance_cfg(d) for d in instances])
    run = pic_run_cfg()
    run.mode, run.n_instances = int(mode), n
    run.tile_r, run.tile_z, run.halo = tile_r, tile_z, halo
    run.sort_interval, run.chunk, run.use_graph = sort_interval, chunk, use_graph
    run.device = device
    run.capacity_factor, run.capacity_min = float(capacity_factor), int(capacity_min)
    run.lanes = int(lanes)
    keep = []
    if use_torch:
        import torch
        torch.cuda.set_device(device)
        s = stream if stream is not None else torch.cuda.current_stream(device)
        run.stream = C.c_void_p(s.cuda_stream)
        al = _TorchAllocator(device, s)
        run.alloc = al.struct()
        keep += [al, s]
    elif stream is not None:
        run.stream = C.c_void_p(stream)
    ctx = C.c_void_p()
    _check(lib().pic_init(C.byref(run), arr, C.byref(ctx)))
    return ctx, keep


def pic_step(ctx, n_steps=1):
    return _check(lib().pic_step(ctx, int(n_steps)), ctx)


def pic_sync(ctx):
    return _check(lib().pic_sync(ctx), ctx)


def pic_destroy(ctx):
    return _check(lib().pic_destroy(ctx))


def pic_last_error(ctx=None):
    m = lib().pic_last_error(ctx)
    return m.decode() if m else ""


def pic_diag(ctx, inst, nodes=None, want_density=False):
    out = pic_diag_t()
    dens = avg = None
    if want_density:
        dens = np.zeros(nodes)
        avg = np.zeros(nodes)
    st = lib().pic_diag(ctx, int(inst), C.byref(out),
                        dens.ctypes.data_as(_D) if dens is not None else None,
                        avg.ctypes.data_as(_D) if avg is not None else None)
    if st not in (PIC_OK, PIC_ECAPACITY, PIC_EOVERFLOW, PIC_ENONFINITE):
        _check(st, ctx)
    d = {}
    for name, _ in pic_diag_t._fields_:
        v = getattr(out, name)
        d[name] = list(v) if hasattr(v, "__len__") else v
    d["status"] = st
    if want_density:
        d["density"], d["time_avg_density"] = dens, avg
    return d


def pic_get_particles(ctx, inst, cap):
    a = [np.zeros(cap) for _ in range(6)]
    key = np.zeros(cap, dtype=np.uint64)
    n = C.c_longlong()
    st = lib().pic_get_particles(ctx, int(inst), *[x.ctypes.data_as(_D) for x in a],
                                 key.ctypes.data_as(_ULL), int(cap), C.byref(n))
    if st not in (PIC_OK, PIC_ECAPACITY, PIC_ENONFINITE):
        _check(st, ctx)
    m = n.value
    out = dict(zip(("r", "z", "vr", "vt", "vz", "w"), [x[:m] for x in a]))
    out["key"] = key[:m]
    return out


def pic_set_particles(ctx, inst, st):
    n = len(st["r"])
    arrs = [np.ascontiguousarray(st[k], dtype=np.float64) for k in ("r", "z", "vr", "vt", "vz", "w")]
    key = np.ascontiguousarray(st["key"], dtype=np.uint64)
    _check(lib().pic_set_particles(ctx, int(inst), n, *[x.ctypes.data_as(_D) for x in arrs],
                                   key.ctypes.data_as(_ULL)), ctx)


def pic_set_fields(ctx, inst, Er=None, Ez=None, Br=None, Bz=None, frozen=1):
    keep = []

    def p(a):
        if a is None:
            return None
        a = np.ascontiguousarray(a, dtype=np.float64).reshape(-1)
        keep.append(a)
        return a.ctypes.data_as(_D)

    _check(lib().pic_set_fields(ctx, int(inst), p(Er), p(Ez), p(Br), p(Bz), int(frozen)), ctx)


def pic_get_fields(ctx, inst, nodes):
    a = [np.zeros(nodes) for _ in range(4)]
    _check(lib().pic_get_fields(ctx, int(inst), *[x.ctypes.data_as(_D) for x in a]), ctx)
    return dict(zip(("Er", "Ez", "Br", "Bz"), a))


def pic_get_charge(ctx, inst, nodes):
    Q = np.zeros(nodes, dtype=np.int64)
    _check(lib().pic_get_charge(ctx, int(inst), Q.ctypes.data_as(_LL)), ctx)
    return Q


def pic_set_cross_sections(ctx, inst, E=None, sigma_el=None, sigma_iz=None):
    if E is None:
        _check(lib().pic_set_cross_sections(ctx, int(inst), 0, None, None, None), ctx)
        return
    a = [np.ascontiguousarray(x, dtype=np.float64) for x in (E, sigma_el, sigma_iz)]
    _check(lib().pic_set_cross_sections(ctx, int(inst), len(a[0]), *[x.ctypes.data_as(_D) for x in a]), ctx)


def pic_set_anisotropy(ctx, inst, E=None, xi=None):
    if E is None:
        _check(lib().pic_set_anisotropy(ctx, int(inst), 0, None, None), ctx)
        return
    a = [np.ascontiguousarray(x, dtype=np.float64) for x in (E, xi)]
    _check(lib().pic_set_anisotropy(ctx, int(inst), len(a[0]), *[x.ctypes.data_as(_D) for x in a]), ctx)


def pic_get_spline3(ctx, inst, nr, nz):
    n = (nr + 3) * (nz + 3)
    Qx = np.zeros(n, dtype=np.int64)
    cx = np.zeros(n)
    _check(lib().pic_get_spline3(ctx, int(inst), Qx.ctypes.data_as(_LL), cx.ctypes.data_as(_D)), ctx)
    return Qx.reshape(nr + 3, nz + 3), cx.reshape(nr + 3, nz + 3)


def pic_get_band_charge(ctx, inst, nodes):
    Qw = np.zeros(nodes, dtype=np.int64)
    _check(lib().pic_get_band_charge(ctx, int(inst), Qw.ctypes.data_as(_LL)), ctx)
    return Qw


def pic_get_phi(ctx, inst, nodes):
    phi = np.zeros(nodes)
    _check(lib().pic_get_phi(ctx, int(inst), phi.ctypes.data_as(_D)), ctx)
    return phi


def pic_set_step(ctx, step):
    return _check(lib().pic_set_step(ctx, int(step)), ctx)


def pic_timing(ctx, enable):
    n = C.c_longlong()
    ms = C.c_double()
    _check(lib().pic_timing(ctx, int(enable), C.byref(n), C.byref(ms)), ctx)
    return n.value, ms.value


def pic_tuning(ctx):
    v = [C.c_int() for _ in range(7)]
    _check(lib().pic_tuning(ctx, *[C.byref(x) for x in v]), ctx)
    return dict(zip(("tile_r", "tile_z", "halo", "sort_interval", "chunk", "lanes", "use_graph"),
                    [x.value for x in v]))


def pic_retune(ctx, tile_r=0, tile_z=0, halo=-1, sort_interval=0):
    return _check(lib().pic_retune(ctx, int(tile_r), int(tile_z), int(halo), int(sort_interval)), ctx)


def pic_autotune(ctx, trial_steps=16, cache_path=None):
    v = [C.c_int() for _ in range(4)]
    ms = C.c_double()
    trials = C.c_int()
    path = cache_path.encode() if cache_path else None
    _check(lib().pic_autotune(ctx, int(trial_steps), path, *[C.byref(x) for x in v], C.byref(ms),
                              C.byref(trials)), ctx)
    out = dict(zip(("tile_r", "tile_z", "halo", "sort_interval"), [x.value for x in v]))
    out["ms_per_step"] = ms.value
    out["trials"] = trials.value
    return out


def pic_reserve(ctx, inst, slots):
    return _check(lib().pic_reserve(ctx, int(inst), int(slots)), ctx)


def pic_capacity(ctx, inst):
    slots = C.c_longlong()
    grows = C.c_longlong()
    _check(lib().pic_capacity(ctx, int(inst), C.byref(slots), C.byref(grows)), ctx)
    return slots.value, grows.value


def pic_moments(ctx, inst, nodes):
    out = np.zeros(11 * nodes)
    _check(lib().pic_moments(ctx, int(inst), out.ctypes.data_as(_D)), ctx)
    return out


def pic_moments_noalloc(ctx, inst, out_ptr):
    """The moments into a caller-owned device array (address out_ptr, 11 x
    nodes doubles), queued on the context's stream; nothing is allocated."""
    _check(lib().pic_moments_noalloc(ctx, int(inst), C.c_void_p(int(out_ptr))), ctx)


def pic_well_depth(ctx, inst, r_mid):
    r = np.ascontiguousarray(r_mid, dtype=np.float64)
    dep = np.zeros(len(r))
    zm = np.zeros(len(r))
    _check(lib().pic_well_depth(ctx, int(inst), len(r), r.ctypes.data_as(_D), dep.ctypes.data_as(_D),
                                zm.ctypes.data_as(_D)), ctx)
    return dep, zm


class Sim:
    """Convenience holder of one context and its instance list."""

    def __init__(self, instances, mode=PIC_MODE_FP64_PLAIN, **kw):
        self.instances = [dict(d) for d in instances]
        self.mode = mode
        self.ctx, self._keep = pic_init(self.instances, mode=mode, **kw)
        self.shapes = [(d["nr"] + 1, d["nz"] + 1) for d in self.instances]

    def nodes(self, k=0):
        return self.shapes[k][0] * self.shapes[k][1]

    def close(self):
        if self.ctx is not None and self.ctx.value:
            pic_destroy(self.ctx)
        self.ctx = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def step(self, n=1):
        pic_step(self.ctx, n)

    def diag(self, k=0, want_density=False):
        d = pic_diag(self.ctx, k, self.nodes(k), want_density)
        if want_density:
            d["density"] = d["density"].reshape(self.shapes[k])
            d["time_avg_density"] = d["time_avg_density"].reshape(self.shapes[k])
        return d

    def get_particles(self, k=0):
        n = self.diag(k)["n_live"]
        return pic_get_particles(self.ctx, k, max(int(n), 1))

    def set_particles(self, st, k=0):
        pic_set_particles(self.ctx, k, st)

    def set_fields(self, k=0, frozen=1, **f):
        pic_set_fields(self.ctx, k, frozen=frozen, **f)

    def fields(self, k=0):
        return {a: v.reshape(self.shapes[k]) for a, v in pic_get_fields(self.ctx, k, self.nodes(k)).items()}

    def charge(self, k=0):
        return pic_get_charge(self.ctx, k, self.nodes(k)).reshape(self.shapes[k])

    def set_cross_sections(self, k=0, E=None, sigma_el=None, sigma_iz=None):
        pic_set_cross_sections(self.ctx, k, E, sigma_el, sigma_iz)

    def set_anisotropy(self, k=0, E=None, xi=None):
        pic_set_anisotropy(self.ctx, k, E, xi)

    def spline3(self, k=0):
        d = self.instances[k]
        return pic_get_spline3(self.ctx, k, d["nr"], d["nz"])

    def band_charge(self, k=0):
        """Band charges of the insert: a node array with bilinear shapes, the
        ghosted (nr+3, nz+3) grid of pic_get_spline3 with cubic shapes."""
        d = self.instances[k]
        if d.get("spline_order", 1) == 3:
            shape = (d["nr"] + 3, d["nz"] + 3)
            return pic_get_band_charge(self.ctx, k, shape[0] * shape[1]).reshape(shape)
        return pic_get_band_charge(self.ctx, k, self.nodes(k)).reshape(self.shapes[k])

    def phi(self, k=0):
        return pic_get_phi(self.ctx, k, self.nodes(k)).reshape(self.shapes[k])

    def set_step(self, step):
        pic_set_step(self.ctx, step)

    def autotune(self, trial_steps=16, cache_path=None):
        return pic_autotune(self.ctx, trial_steps, cache_path)

    def retune(self, **kw):
        pic_retune(self.ctx, **kw)

    def moments(self, k=0):
        """(11, nr+1, nz+1): n, n u_r, n u_t, n u_z, second moments (rr, rt, rz,
        tt, tz, zz), sum w nu_m / V."""
        return pic_moments(self.ctx, k, self.nodes(k)).reshape((11,) + self.shapes[k])

    def well_depth(self, r_mid, k=0):
        return pic_well_depth(self.ctx, k, r_mid)

    def capacity(self, k=0):
        return pic_capacity(self.ctx, k)

    def reserve(self, slots, k=0):
        pic_reserve(self.ctx, k, slots)
