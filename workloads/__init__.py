"""Seeded synthetic workloads shaped like the paper's runs.

This module is the only thing the oracle and the HIP path share.  It holds
configuration dictionaries and seeded random states and none of the method's
arithmetic: no field solve, push, deposit, rate, probability or unit
conversion of the method happens here.

Configuration dictionary (both sides read the same keys):
  ndim, n[ndim] (cells), dx[ndim] (m), cfl, nsteps, transverse_bc
  ("outflow" | "periodic"), materials (list of dicts: gap_eV, n_index,
  density_gcc, molar_mass_gmol, me_star, mh_star, pos_mass_kg, and for a
  single-pole Lorentz response lorentz_lambda_m, eps_inf, lorentz_gamma_s; for
  impact ionization impact_rate_s; for the Kerr response kerr_n2_m2W), layers (list
  of (material, lo_m, hi_m) half-open along x), ppc, T_K, shape_order,
  keldysh_terms, seed, laser (lambda_m, fwhm_s, peak_Wcm2 | fluence_Jcm2,
  waist_m, t_peak_s, cep_rad, envelope "gauss" | "sin2", pol_axis),
  particle_capacity, preionize_eV (0 = off; >0: every neutral starts ionized,
  carriers thermal at that temperature -- the charged-loop stress variant),
  collisions (optional, default off: binary collisions among the charged
  particles).

The paper's runs (Sec. 3) are 3D with ~1e10 macroparticles and are not
reproduced; the configurations below are the synthetic stand-ins the
benchmark and parity tests use, with the paper's materials (Table 1), pulse
shapes (Sec. 3) and mirror geometry (Fig. 1) where they apply.
"""

import numpy as np

LAMBDA = 800e-9
_C = 299792458.0      # only to express "N optical cycles" as a duration


def cycles(n, lam=LAMBDA):
    return n * lam / _C


def silica_like():
    """The n = 1.45, 9 eV material of the benchmark configurations (SiO2 masses)."""
    return dict(gap_eV=9.0, n_index=1.45, density_gcc=2.2, molar_mass_gmol=60.08,
                me_star=0.6, mh_star=8.0, pos_mass_kg=0.0)


def high_index():
    """The n = 2.1, 4 eV material of the mirror configuration (HfO2 masses, density)."""
    return dict(gap_eV=4.0, n_index=2.1, density_gcc=9.68, molar_mass_gmol=210.49,
                me_star=1.09, mh_star=1.12, pos_mass_kg=0.0)


def table1_sio2():
    """Fused silica as listed in the paper's Table 1."""
    return dict(gap_eV=9.0, n_index=1.477, density_gcc=2.2, molar_mass_gmol=60.08,
                me_star=0.6, mh_star=8.0, pos_mass_kg=0.0)


def table1_hfo2():
    """HfO2 as listed in the paper's Table 1."""
    return dict(gap_eV=5.7, n_index=2.021, density_gcc=9.68, molar_mass_gmol=210.49,
                me_star=1.09, mh_star=1.12, pos_mass_kg=0.0)


def lorentz(mat, lambda0_m, eps_inf=1.0, gamma_s=0.0):
    """The material with a single-pole Lorentz response: resonance at the
    wavelength lambda0_m, instantaneous permittivity eps_inf, damping rate
    gamma_s [1/s].  n_index stays the index at the laser wavelength."""
    return dict(mat, lorentz_lambda_m=lambda0_m, eps_inf=eps_inf, lorentz_gamma_s=gamma_s)


# Dispersive variants: one ultraviolet pole per material, the deeper
# ultraviolet response folded into eps_inf (fused silica: the pole near
# 0.116 um of its Sellmeier fit, eps_inf = 1 + the 0.068 um term's strength;
# HfO2: a pole at 0.15 um, eps_inf = 2)
SILICA_UV = (0.116e-6, 1.7)
HFO2_UV = (0.15e-6, 2.0)


def silica_dispersive():
    return lorentz(silica_like(), SILICA_UV[0], eps_inf=SILICA_UV[1])


def high_index_dispersive():
    return lorentz(high_index(), HFO2_UV[0], eps_inf=HFO2_UV[1])


def with_impact(mat, rate_s):
    """The material with impact ionization at Keldysh's rate constant rate_s [1/s]."""
    return dict(mat, impact_rate_s=rate_s)


def layer_stack(mats, n_indices, x0, lam=LAMBDA, first_half_wave=False):
    """Quarter-wave stack (Fig. 1): each layer lam/(4n); optionally the first
    (protective) layer lam/(2n).  Returns [(mat, lo, hi), ...] starting at x0."""
    out = []
    x = x0
    for i, (m, n) in enumerate(zip(mats, n_indices)):
        t = lam / ((2.0 if (first_half_wave and i == 0) else 4.0) * n)
        out.append((m, x, x + t))
        x += t
    return out


def _laser(cyc, peak=0.0, fluence=0.0, waist=0.0, env="gauss"):
    return dict(lambda_m=LAMBDA, fwhm_s=cycles(cyc), peak_Wcm2=peak, fluence_Jcm2=fluence,
                waist_m=waist, t_peak_s=0.0, cep_rad=0.0, envelope=env, pol_axis=1)


def config_1d(hi=False, nsteps=2000, n=1024, ppc=100, peak=None, dispersive=False):
    """1D3V slab: 1024 cells at lambda/40, n = 1.45 slab over cells 400-600,
    2-cycle Gaussian pulse at 1e13 W/cm^2 (1e14 for the high-intensity variant,
    which ionizes enough to exercise the Monte-Carlo step), seed 0.
    dispersive: the slab responds as a Lorentz medium (index 1.45 at 800 nm)."""
    dx = LAMBDA / 40
    mat = silica_dispersive() if dispersive else silica_like()
    pk = peak if peak is not None else (1e14 if hi else 1e13)
    lo = int(round(n * 400 / 1024))
    hi_c = int(round(n * 600 / 1024))
    return dict(ndim=1, n=[n], dx=[dx], cfl=0.95, nsteps=nsteps, transverse_bc="outflow",
                materials=[mat], layers=[(0, lo * dx, hi_c * dx)], ppc=ppc,
                T_K=300.0, shape_order=2, keldysh_terms=500, seed=0,
                laser=_laser(2, peak=pk), particle_capacity=0, preionize_eV=0.0)


def config_2d(nx=2048, ny=512, nsteps=4000, ppc=16, peak=5e13, seed=1, slab_cells=80,
              front=None, waist=3e-6, bc="outflow", dispersive=False):
    """2D3V slab: 2048 x 512 cells at lambda/32, 2 um silica-like slab filling y,
    16 neutrals per cell, 3-cycle pulse, waist 3 um, 5e13 W/cm^2, seed 1.
    dispersive: the slab responds as a Lorentz medium."""
    dx = LAMBDA / 32
    mat = silica_dispersive() if dispersive else silica_like()
    f = nx // 4 if front is None else front
    return dict(ndim=2, n=[nx, ny], dx=[dx, dx], cfl=0.95, nsteps=nsteps, transverse_bc=bc,
                materials=[mat], layers=[(0, f * dx, (f + slab_cells) * dx)], ppc=ppc,
                T_K=300.0, shape_order=2, keldysh_terms=500, seed=seed,
                laser=_laser(3, peak=peak, waist=waist), particle_capacity=0, preionize_eV=0.0)


def config_3d(nx=256, ny=128, nz=128, nsteps=2000, ppc=8, fluence=1.0, seed=2, front=64,
              dispersive=False):
    """3D3V one-GPU share of a multi-layer mirror: 256 x 128 x 128 cells at
    lambda/24, 8 alternating quarter-wave layers (n = 1.45, 9 eV / n = 2.1,
    4 eV), 8 neutrals per cell, 2-cycle plane-wave pulse of 1 J/cm^2, periodic
    transverse boundaries (the neighbours of this share), seed 2.
    dispersive: both layer materials respond as Lorentz media."""
    dx = LAMBDA / 24
    mats = [0, 1] * 4
    m0, m1 = silica_like(), high_index()
    if dispersive:
        m0, m1 = silica_dispersive(), high_index_dispersive()
    layers = layer_stack(mats, [1.45, 2.1] * 4, front * dx)
    return dict(ndim=3, n=[nx, ny, nz], dx=[dx, dx, dx], cfl=0.95, nsteps=nsteps,
                transverse_bc="periodic", materials=[m0, m1],
                layers=layers, ppc=ppc, T_K=300.0, shape_order=2, keldysh_terms=500,
                seed=seed, laser=_laser(2, fluence=fluence), particle_capacity=0,
                preionize_eV=0.0)


def config_stress(base, eV=2.0):
    """Charged-loop stress variant: every neutral starts ionized, carriers thermal."""
    c = dict(base)
    c["preionize_eV"] = eV
    return c


def batch_scan(n_inst=32, nsteps=3000):
    """Fluence scan: 32 independent 2D3V instances, grids 256x128 .. 1536x512,
    fluences log-spaced 0.05 .. 3 J/cm^2, slab 0.5 .. 3 um, 8 .. 32 ppc,
    seeds 100 .. 131."""
    out = []
    dx = LAMBDA / 32
    for i in range(n_inst):
        rng = np.random.default_rng(100 + i)
        nx = int(rng.choice([256, 512, 768, 1024, 1280, 1536]))
        ny = int(rng.choice([128, 256, 384, 512]))
        thick = float(rng.uniform(0.5e-6, 3e-6))
        ppc = int(rng.choice([8, 16, 24, 32]))
        F = 0.05 * 60.0 ** (i / max(n_inst - 1, 1))
        slab = max(1, int(round(thick / dx)))
        front = nx // 4
        slab = min(slab, nx - front - 8)
        c = dict(ndim=2, n=[nx, ny], dx=[dx, dx], cfl=0.95, nsteps=nsteps,
                 transverse_bc="outflow", materials=[silica_like()],
                 layers=[(0, front * dx, (front + slab) * dx)], ppc=ppc, T_K=300.0,
                 shape_order=2, keldysh_terms=500, seed=100 + i,
                 laser=_laser(3, fluence=F, waist=3e-6), particle_capacity=0, preionize_eV=0.0)
        out.append(c)
    return out


def served_requests(n_req=400, rate_hz=4.0, seed=7, scale=1.0):
    """Poisson arrivals of mixed 1D / 2D / 3D runs with random fluence
    (log-uniform 0.05 .. 3 J/cm^2) and 1 .. 8 mirror layers.  ``scale`` < 1
    shrinks grids and step counts for short rehearsals."""
    rng = np.random.default_rng(seed)
    t = 0.0
    reqs = []
    for i in range(n_req):
        t += rng.exponential(1.0 / rate_hz)
        kind = int(rng.integers(0, 3))
        F = float(np.exp(rng.uniform(np.log(0.05), np.log(3.0))))
        nl = int(rng.integers(1, 9))
        mats = [i_ % 2 for i_ in range(nl)]
        ns = [1.45 if m == 0 else 2.1 for m in mats]
        if kind == 0:
            nx = int(rng.integers(1024, 8193) * scale)
            dx = LAMBDA / 40
            steps = int(2000 * scale)
            c = dict(ndim=1, n=[nx], dx=[dx], cfl=0.95, nsteps=steps, transverse_bc="outflow",
                     ppc=max(1, int(100 * scale)))
        elif kind == 1:
            nx = int(rng.integers(256, 1025) * scale)
            ny = int(rng.integers(64, 513) * scale)
            dx = LAMBDA / 32
            steps = int(3000 * scale)
            c = dict(ndim=2, n=[nx, ny], dx=[dx, dx], cfl=0.95, nsteps=steps,
                     transverse_bc="outflow", ppc=16)
        else:
            m = int(rng.integers(32, 129) * scale)
            nx = max(m, 64)
            dx = LAMBDA / 24
            steps = int(2000 * scale)
            c = dict(ndim=3, n=[nx, max(8, m // 2), max(8, m // 2)], dx=[dx, dx, dx], cfl=0.95,
                     nsteps=steps, transverse_bc="periodic", ppc=8)
        front = c["n"][0] // 4
        layers = layer_stack(mats, ns, front * dx)
        # keep the stack inside the box
        layers = [L for L in layers if L[2] < (c["n"][0] - 8) * dx] or [layers[0]]
        c.update(materials=[silica_like(), high_index()], layers=layers, T_K=300.0,
                 shape_order=2, keldysh_terms=500, seed=1000 + i,
                 laser=_laser(2, fluence=F, waist=0.0), particle_capacity=0, preionize_eV=0.0)
        reqs.append(dict(arrival_s=t, cfg=c))
    return reqs


def domain_shape(cfg, which, comp):
    """Shape (nx', ny', nz') of field component ``comp`` of ``which`` ('E'|'b')
    on its own staggered positions inside the box (no guards)."""
    D = cfg["ndim"]
    per = cfg.get("transverse_bc", "outflow") == "periodic"
    out = []
    for d in range(3):
        if d >= D:
            out.append(1)
            continue
        n = cfg["n"][d]
        half = (d == comp) if which == "E" else (d != comp)
        periodic = per and d > 0
        out.append(n if (half or periodic) else n + 1)
    return tuple(out)


def random_state(cfg, n_particles, seed, e_scale=3e10, u_scale=0.3, margin=3.0):
    """A seeded random mid-run state for one-step parity tests: E and b on every
    in-box position, charged particles (cell, offset, u, kind) away from the
    outflow faces by ``margin`` cells.  Offsets are FP32 numbers in [0, 1)."""
    rng = np.random.default_rng(seed)
    D = cfg["ndim"]
    E = [rng.uniform(-e_scale, e_scale, domain_shape(cfg, "E", c)) for c in range(3)]
    b = [rng.uniform(-e_scale, e_scale, domain_shape(cfg, "b", c)) for c in range(3)]
    per = cfg.get("transverse_bc", "outflow") == "periodic"
    cell = np.zeros((n_particles, 3), dtype=np.int64)
    off = np.zeros((n_particles, 3), dtype=np.float32)
    for d in range(D):
        n = cfg["n"][d]
        m = 0 if (per and d > 0) else int(margin)
        cell[:, d] = rng.integers(m, n - m, n_particles)
        off[:, d] = rng.integers(0, 2 ** 24, n_particles).astype(np.float32) * np.float32(2.0 ** -24)
    u = rng.normal(0.0, u_scale, (n_particles, 3))
    nk = 2 * len(cfg["materials"])
    kind = rng.integers(0, nk, n_particles)
    return dict(E=E, b=b, cell=cell, off=off, u=u, kind=kind)


def face_state(cfg, n_per_face, seed, e_scale=1e9, u_out=(0.3, 2.0)):
    """A seeded state with charged particles in the cells next to every outflow
    face (x faces always; y, z faces when the transverse boundaries are
    outflow), each moving outward with |u| along the face normal drawn from
    ``u_out`` and random transverse components, so that they leave the box
    within a few steps; E and b random on every in-box position."""
    rng = np.random.default_rng(seed)
    D = cfg["ndim"]
    per = cfg.get("transverse_bc", "outflow") == "periodic"
    E = [rng.uniform(-e_scale, e_scale, domain_shape(cfg, "E", c)) for c in range(3)]
    b = [rng.uniform(-e_scale, e_scale, domain_shape(cfg, "b", c)) for c in range(3)]
    cells, offs, us = [], [], []
    for d in range(D):
        if per and d > 0:
            continue
        for side in (0, 1):
            cell = np.zeros((n_per_face, 3), dtype=np.int64)
            for e in range(D):
                cell[:, e] = rng.integers(0, cfg["n"][e], n_per_face)
            cell[:, d] = 0 if side == 0 else cfg["n"][d] - 1
            off = np.zeros((n_per_face, 3), dtype=np.float32)
            for e in range(D):
                off[:, e] = rng.integers(0, 2 ** 24, n_per_face).astype(np.float32) * np.float32(2.0 ** -24)
            u = rng.normal(0.0, 0.2, (n_per_face, 3))
            u[:, d] = rng.uniform(u_out[0], u_out[1], n_per_face) * (-1.0 if side == 0 else 1.0)
            cells.append(cell)
            offs.append(off)
            us.append(u)
    cell = np.concatenate(cells)
    nk = 2 * len(cfg["materials"])
    kind = rng.integers(0, nk, len(cell))
    return dict(E=E, b=b, cell=cell, off=np.concatenate(offs), u=np.concatenate(us), kind=kind)
