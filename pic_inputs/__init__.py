"""Seeded synthetic inputs shared by the tests, the benchmark and the oracle
wrapper.

This module only holds parameter values and seeded random states.  It holds
none of the method's arithmetic (no derived constants, no push, no deposit),
so both the HIP path and the oracle can take their inputs from it without
sharing any computation.

Workloads (coaxial trap, Sec. II.B of the paper for the structure: coaxial
electrodes with an applied bias, axial B ~ 0.28 T, uniform neutral gas,
Maxwellian 1 eV seed cloud as in Sec. III.A).  The paper's own geometry,
Ne cross-section tables and field map are not available, so these synthetic
coaxial traps stand in for them:

    coax64     64x128 mesh, 1 instance, 50k electrons, uniform B      (FP64)
    coax64hot  the same at 1e-1 mbar, the paper's raised pressure    (FP64)
    coax256    256x1024 mesh, 4M electrons, mirror B, 1e-5 mbar      (FP64)
    coax512    512x2048 mesh, 64M electrons, mirror B, -30 kV        (FP32)
    scan32     32 instances on 128x512, p/V/B scan, 0.5M-8M each     (FP32)
    batch8     8 instances on 256x1024, 16M each, mirror B           (FP32)
    gun        the paper's own geometry: coax with the elliptic insert, open
               ends, 30 kV, 64x128 mesh (both forms)
    gun8       8 gun instances on 256x512, 16M each                  (FP32)
"""
import math

import numpy as np

# Electrode geometry and the common trap parameters.
_BASE = dict(
    a=1.0e-3, b=10.0e-3, L=60.0e-3, nr=64, nz=128,
    V_inner=-20000.0, V_outer=0.0, V_end=-2000.0, end_mode=0,
    B0=0.28, mirror_k=0.0,
    p_mbar=1.0e-6, T_gas_K=300.0, M_gas_amu=2.016,
    sigma_el=1.0e-19, iz_I_eV=15.4, lotz_a=4.5e-18, lotz_q=2.0,
    opal_Ebar_eV=10.0, okh_xi=0.0, E_cap_eV=0.0,
    n_init=50000, r_lo=3.0e-3, r_hi=7.0e-3, z_lo=20.0e-3, z_hi=40.0e-3,
    T_init_eV=1.0, weight=1.0e5, load_mode=1,
    seed=0, dt=1.0e-12, fx_shift=0, diag_interval=10, collisions=1,
    src_rate=0.0, src_T_eV=0.0,
    ins_r0=0.0, ins_z0=0.0, ins_er=0.0, ins_ez=0.0, ins_band=0.0, spline_order=1, okh_E0_eV=0.0,
)

# Total seed charge of the small case (50k x 1e5 electrons) is kept for the
# larger particle counts, so the initial density stays ~2e15 m^-3 rather than
# exceeding the Brillouin limit eps0 B^2 / (2 m_e) at 0.28 T.
_SEED_ELECTRONS = 5.0e9


def e_cap(cfg):
    """Energy bound (eV) for the null-collision rate: 1.1 x the largest
    potential difference in the trap plus 20 T_init."""
    span = abs(cfg["V_inner"] - cfg["V_outer"]) + abs(cfg["V_end"])
    return 1.1 * span + 20.0 * cfg["T_init_eV"]


def _finish(cfg):
    cfg = dict(cfg)
    if cfg["E_cap_eV"] <= 0.0:
        cfg["E_cap_eV"] = e_cap(cfg)
    return cfg


def coax64(**over):
    c = dict(_BASE)
    c.update(over)
    return _finish(c)


def coax64hot(**over):
    return coax64(p_mbar=1.0e-1, **over)


def coax256(**over):
    c = dict(_BASE, nr=256, nz=1024, n_init=4_000_000, mirror_k=0.3, p_mbar=1.0e-5,
             weight=_SEED_ELECTRONS / 4.0e6, seed=1)
    c.update(over)
    return _finish(c)


def coax512(**over):
    c = dict(_BASE, nr=512, nz=2048, n_init=64_000_000, mirror_k=0.3, V_inner=-30000.0,
             p_mbar=1.0e-6, weight=_SEED_ELECTRONS / 64.0e6, seed=2)
    c.update(over)
    return _finish(c)


def scan32(n_scale=1.0):
    """32-instance parameter scan: pressure log-spaced 1e-7..1e-5 mbar, inner
    voltage -15..-30 kV and B0 0.2..0.35 T linearly spaced but permuted
    (7i mod 32 and 13i mod 32) so the three axes are decorrelated; particle
    counts log-uniform over 0.5M..8M from a seeded generator."""
    rng = np.random.default_rng(3)
    n = rng.uniform(math.log(0.5e6), math.log(8e6), size=32)
    out = []
    for i in range(32):
        p = 1.0e-7 * 100.0 ** (i / 31.0)
        V = -15000.0 - 15000.0 * ((7 * i) % 32) / 31.0
        B = 0.20 + 0.15 * ((13 * i) % 32) / 31.0
        N = max(1, int(round(math.exp(n[i]) * n_scale)))
        c = dict(_BASE, nr=128, nz=512, p_mbar=p, V_inner=V, B0=B, mirror_k=0.0, n_init=N,
                 weight=_SEED_ELECTRONS / N, seed=(3 << 32) | i)
        out.append(_finish(c))
    return out


def batch8(n_per=16_000_000):
    """8 instances on 256x1024 meshes, 16M electrons each, mirror field,
    pressures cycling 1e-6, 3e-6, 1e-5 mbar."""
    press = (1.0e-6, 3.0e-6, 1.0e-5)
    out = []
    for i in range(8):
        c = dict(_BASE, nr=256, nz=1024, n_init=n_per, mirror_k=0.3, p_mbar=press[i % 3],
                 weight=_SEED_ELECTRONS / n_per, seed=(4 << 32) | i)
        out.append(_finish(c))
    return out


def gun(**over):
    """The paper's geometry (Sec. III, the corona-ring region of the gun): a
    coax with r_a = 63.75 mm and r_b = 81 mm between open ends (d(phi)/dz = 0)
    at z = -10 mm and 34 mm, here shifted to 0 .. 44 mm, with a filled
    elliptic insert on the outer cylinder centred at r = 81 mm, z = 12 mm
    (here 22 mm), semi-axes 3 mm in r and 14 mm in z.  Bias 30 kV (inner
    conductor at -30 kV), B ~ 0.28 T (uniform here: the paper's field map is
    not available), the raised pressure 1e-1 mbar, a 1 eV seed cloud of
    ~1e15 m^-3 in a load box clear of the insert (Sec. III.A)."""
    c = dict(_BASE, a=63.75e-3, b=81.0e-3, L=44.0e-3, nr=64, nz=128,
             V_inner=-30000.0, V_outer=0.0, V_end=0.0, end_mode=2, B0=0.28, mirror_k=0.0,
             p_mbar=1.0e-1, n_init=50000, r_lo=66.0e-3, r_hi=76.0e-3, z_lo=2.0e-3, z_hi=42.0e-3,
             load_mode=0, weight=3.6e6, seed=5,
             ins_r0=81.0e-3, ins_z0=22.0e-3, ins_er=3.0e-3, ins_ez=14.0e-3)
    c.update(over)
    return _finish(c)


def gun8(n_per=16_000_000, nr=256, nz=512):
    """8 gun instances (pressures 2.5e-2 .. 1e-1 mbar and biases 20 .. 40 kV)
    on nr x nz meshes, n_per electrons each, the seed weight kept at the
    1e15 m^-3 density of the small case."""
    out = []
    press = (2.5e-2, 5.0e-2, 1.0e-1, 1.0e-1)
    bias = (-30000.0, -30000.0, -30000.0, -20000.0, -40000.0)
    for i in range(8):
        out.append(gun(nr=nr, nz=nz, n_init=n_per, weight=3.6e6 * 50000 / n_per, p_mbar=press[i % 4],
                       V_inner=bias[i % 5], E_cap_eV=0.0, seed=(6 << 32) | i))
    return out


def synthetic_xs(cfg, n=200, E_max=1.0e5):
    """A synthetic cross-section table in LXCat layout (the paper's Ne data
    are not available): n log-spaced energies 1e-2 .. E_max eV, an elastic
    momentum-transfer cross section falling from ~2e-19 m^2 at low energy to
    ~2e-21 m^2 at 10 keV, and an ionisation cross section that is zero up to
    the configuration's threshold, peaks at 1e-20 m^2 at 100 eV above it and
    falls as 1/E beyond (a plain rational curve, not a physics model)."""
    E = np.geomspace(1.0e-2, E_max, n)
    el = 2.0e-19 / (1.0 + E / 50.0) ** 0.75 + 2.0e-22
    t = np.maximum(E - cfg["iz_I_eV"], 0.0) / 100.0
    iz = 4.0e-20 * t / (1.0 + t) ** 2
    return E, el, iz


WORKLOADS = {
    "coax64": lambda: [coax64()],
    "coax64hot": lambda: [coax64hot()],
    "coax256": lambda: [coax256()],
    "coax512": lambda: [coax512()],
    "scan32": scan32,
    "batch8": batch8,
    "gun": lambda: [gun()],
    "gun8": gun8,
}


# ---------------------------------------------------------------------------
# Random particle states and prescribed fields for parity tests
# ---------------------------------------------------------------------------

def particle_state(cfg, n, seed, v_scale=1.0e6, margin_cells=0.5, key_base=0):
    """n particles spread over the whole mesh (not just the load box), with
    velocity components normal with std v_scale; keys key_base..key_base+n-1.
    Positions stay margin_cells cells away from the walls."""
    rng = np.random.default_rng(seed)
    dr = (cfg["b"] - cfg["a"]) / cfg["nr"]
    dz = cfg["L"] / cfg["nz"]
    r = rng.uniform(cfg["a"] + margin_cells * dr, cfg["b"] - margin_cells * dr, n)
    z = rng.uniform(margin_cells * dz, cfg["L"] - margin_cells * dz, n)
    vr = rng.normal(0.0, v_scale, n)
    vt = rng.normal(0.0, v_scale, n)
    vz = rng.normal(0.0, v_scale, n)
    w = np.full(n, float(cfg["weight"]))
    key = np.arange(key_base, key_base + n, dtype=np.uint64)
    return dict(r=r, z=z, vr=vr, vt=vt, vz=vz, w=w, key=key)


def cloud_state(cfg, n, seed, key_base=0):
    """n particles in the load box with speeds spread over 1 eV .. 2 keV, the
    energy range of E x B-drifting electrons in these traps."""
    rng = np.random.default_rng(seed)
    r = rng.uniform(cfg["r_lo"], cfg["r_hi"], n)
    z = rng.uniform(cfg["z_lo"], cfg["z_hi"], n)
    E = np.exp(rng.uniform(math.log(1.0), math.log(2000.0), n))
    speed = np.sqrt(2.0 * E * 1.602176634e-19 / 9.1093837015e-31)
    u = rng.normal(size=(3, n))
    u /= np.linalg.norm(u, axis=0)
    w = np.full(n, float(cfg["weight"]))
    key = np.arange(key_base, key_base + n, dtype=np.uint64)
    return dict(r=r, z=z, vr=speed * u[0], vt=speed * u[1], vz=speed * u[2], w=w, key=key)


def random_fields(cfg, seed, e_scale=2.0e6, b_scale=0.3):
    """Smooth random nodal fields (a few low Fourier modes) for frozen-field
    parity tests; arrays are r-major (nr+1, nz+1)."""
    rng = np.random.default_rng(seed)
    nr, nz = cfg["nr"], cfg["nz"]
    x = np.linspace(0.0, 1.0, nr + 1)[:, None]
    y = np.linspace(0.0, 1.0, nz + 1)[None, :]

    def smooth(scale):
        f = np.zeros((nr + 1, nz + 1))
        for _ in range(4):
            kx, ky = rng.integers(0, 4, 2)
            ph1, ph2 = rng.uniform(0, 2 * math.pi, 2)
            f += rng.normal() * np.cos(math.pi * kx * x + ph1) * np.cos(math.pi * ky * y + ph2)
        return scale * f / 4.0

    return dict(Er=smooth(e_scale), Ez=smooth(e_scale), Br=smooth(0.1 * b_scale),
                Bz=b_scale + smooth(0.2 * b_scale))


def ballistic_state(cfg, groups, v):
    """Electrons moving radially at speed v, for runs with zero fields: group
    (wall, s, n) holds n electrons that start half of a step's flight v dt
    short of s steps from wall 0 (inner, moving inward) or 1 (outer, moving
    outward), spread along z over the middle of the trap."""
    r, vr = [], []
    h = v * cfg["dt"]
    for wall, s, n in groups:
        r += [cfg["b"] - (s - 0.5) * h if wall == 1 else cfg["a"] + (s - 0.5) * h] * n
        vr += [v if wall == 1 else -v] * n
    n = len(r)
    return dict(r=np.array(r), z=np.linspace(0.1 * cfg["L"], 0.9 * cfg["L"], n), vr=np.array(vr),
                vt=np.zeros(n), vz=np.zeros(n), w=np.full(n, cfg["weight"]), key=np.arange(n, dtype=np.uint64))


def uniform_fields(cfg, Er=0.0, Ez=0.0, Br=0.0, Bz=0.0):
    shape = (cfg["nr"] + 1, cfg["nz"] + 1)
    return dict(Er=np.full(shape, float(Er)), Ez=np.full(shape, float(Ez)),
                Br=np.full(shape, float(Br)), Bz=np.full(shape, float(Bz)))
