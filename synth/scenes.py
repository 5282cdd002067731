"""Seeded synthetic scenes shaped like the paper's solar-atmosphere workloads.

The paper's own model (a 2D 512x768 Kelvin-Helmholtz prominence, Sect. 4.1)
and its atomic data are not available, so every input here is synthetic:
Gaussian random fields (GRF) for opacity, temperature and velocity, sparse
brick occupancy, and spectral lines described by the Core-and-Voigt
parameters of Sect. 3.2 (eta*, chi*, damping a, 1/Doppler width, bulk
velocity) plus a grey background.

Conventions shared by every scene dict:
  * index space, MIP-0 voxel side 1; voxel linear index x + nx*(y + ny*z);
  * per-voxel arrays are float32, flattened with x fastest;
  * per-wavelength static arrays are [n_lam][nvox];
  * line arrays are [n_lines][nvox]; velocity is [dim][nvox] in km/s;
  * wavelengths (nm) are float64;
  * directions are float32 unit vectors [n_dir][dim];
  * blocks (bricks) are numbered bx + nbx*(by + nby*bz).

Nothing in this module evaluates a line profile, averages a mip, traverses a
grid or integrates the transfer equation.
"""
from __future__ import annotations

import math

import numpy as np
from scipy.special import ndtr

C_KMS = 299792.458  # speed of light, km/s


# --------------------------------------------------------------------------
# random fields
# --------------------------------------------------------------------------
def grf(rng: np.random.Generator, shape, ell: float) -> np.ndarray:
    """Periodic Gaussian random field with covariance ~ exp(-r^2 / (2 ell^2)).

    White N(0,1) noise filtered in Fourier space by a Gaussian of standard
    deviation ell/sqrt(2) (so the field's correlation length is ell), then
    standardised to sample mean 0 and standard deviation 1.  float64.
    """
    shape = tuple(int(s) for s in shape)
    white = rng.standard_normal(shape)
    sig = ell / math.sqrt(2.0)
    f = np.fft.rfftn(white)
    k2 = np.zeros(f.shape)
    for ax, n in enumerate(shape):
        if ax == len(shape) - 1:
            k = np.fft.rfftfreq(n) * 2.0 * np.pi
        else:
            k = np.fft.fftfreq(n) * 2.0 * np.pi
        sh = [1] * len(shape)
        sh[ax] = k.size
        k2 = k2 + (k.reshape(sh)) ** 2
    f *= np.exp(-0.5 * k2 * sig * sig)
    g = np.fft.irfftn(f, s=shape, axes=tuple(range(len(shape))))
    g -= g.mean()
    sd = g.std()
    if sd > 0:
        g /= sd
    return g


def _tmap(rng, shape, ell):
    """Temperature-like field T = 0.5 + 1.5*Phi(g) in [0.5, 2]."""
    return 0.5 + 1.5 * ndtr(grf(rng, shape, ell))


# --------------------------------------------------------------------------
# directions and ray samples
# --------------------------------------------------------------------------
def directions_2d(n_dir: int) -> np.ndarray:
    """theta_k = 2 pi (k + 1/2) / n_dir, as float32 (cos, sin)."""
    th = 2.0 * np.pi * (np.arange(n_dir) + 0.5) / n_dir
    return np.stack([np.cos(th), np.sin(th)], axis=1).astype(np.float32)


def directions_fibonacci(n_dir: int) -> np.ndarray:
    """Fibonacci-sphere directions: z_i = 1 - 2(i+1/2)/n, phi_i = pi(1+sqrt5) i."""
    i = np.arange(n_dir, dtype=np.float64)
    z = 1.0 - 2.0 * (i + 0.5) / n_dir
    phi = np.pi * (1.0 + math.sqrt(5.0)) * i
    r = np.sqrt(np.maximum(0.0, 1.0 - z * z))
    return np.stack([r * np.cos(phi), r * np.sin(phi), z], axis=1).astype(np.float32)


def _blocks_shape(n, dim, B):
    return tuple(n[a] // B for a in range(dim))


def _mask_from_blocks(n, dim, B, block_active):
    nb = _blocks_shape(n, dim, B)
    act = block_active.reshape(tuple(reversed(nb)))
    m = act
    for ax in range(dim):
        m = np.repeat(m, B, axis=ax)
    return m.astype(bool)  # shape reversed(n[:dim])


def _shape_rev(n, dim):
    return tuple(reversed(n[:dim]))


# --------------------------------------------------------------------------
# configurations
# --------------------------------------------------------------------------
def make_cfg1(seed: int = 1, n: int = 64, B: int = 8, n_empty: int = 19, n_lam: int = 16,
              n_dir: int = 8, ell: float = 6.0):
    """2D static scene: n^2 grid, BxB bricks, n_empty bricks with eta = chi = 0.

    ln chi* = GRF(-2, 1.5, ell); T = 0.5 + 1.5 Phi(GRF(ell_T = 2 ell)); S = exp(-1/T);
    chi(k) = chi* exp(-((k - (n_lam-1)/2)/4)^2) over n_lam wavelength bins
    (a Gaussian line of Doppler width 4 bins), eta = S chi, zero velocity.
    """
    dim = 2
    shp = (n, n)
    ss = np.random.SeedSequence(seed)
    r_chi, r_t, r_e = [np.random.default_rng(s) for s in ss.spawn(3)]
    ln_chi = -2.0 + 1.5 * grf(r_chi, shp, ell)
    T = _tmap(r_t, shp, 2.0 * ell)
    S = np.exp(-1.0 / T)
    nb = (n // B) ** 2
    empty = r_e.choice(nb, size=n_empty, replace=False)
    block_active = np.ones(nb, dtype=np.uint8)
    block_active[empty] = 0
    mask = _mask_from_blocks((n, n, 1), dim, B, block_active)
    k = np.arange(n_lam, dtype=np.float64)
    prof = np.exp(-(((k - 0.5 * (n_lam - 1)) / 4.0) ** 2))
    chi_star = np.exp(ln_chi) * mask
    chi = (prof[:, None, None] * chi_star[None]).astype(np.float32)
    eta = (prof[:, None, None] * (S * chi_star)[None]).astype(np.float32)
    return dict(
        name="cfg1", dim=dim, n=(n, n, 1), brick=B, n_levels=4, model="static",
        eta=eta.reshape(n_lam, -1), chi=chi.reshape(n_lam, -1),
        dirs=directions_2d(n_dir), block_active=block_active, ds0=1.0, I0=0.0,
        iod_threshold=(1e-2, 1.0), tau_thin=0.25, lam_batch=8,
    )


def make_cfg2(seed: int = 2, n: int = 1024, B: int = 16, active_frac: float = 0.4,
              n_lam_per_line: int = 128, n_dir: int = 64, ell: float = 24.0):
    """2D moving-medium line scene (velocity interpolation workload).

    Active bricks: the top active_frac of a brick-level GRF(0,1,4 bricks).
    Two Gaussian lines (lam0 = 500.00, 500.25 nm, thermal width 10 km/s):
    ln chi*_0 = GRF(-2, 1.5, ell), ln chi*_1 = GRF(-4, 1.5, ell); grey
    continuum ln chi_c = GRF(-6, 0.5, 2 ell); eta = S chi with S from a T-map
    (ell_T = 2 ell); velocity (vx, vy) each GRF(0, 12 km/s, 2 ell), rescaled so
    that max |v| = 30 km/s.  n_lam_per_line wavelengths per line, uniform in
    Doppler offset over [-60, 60] km/s.
    """
    dim = 2
    shp = (n, n)
    ss = np.random.SeedSequence(seed)
    rs = [np.random.default_rng(s) for s in ss.spawn(7)]
    nbx = n // B
    g_b = grf(rs[0], (nbx, nbx), 4.0).reshape(-1)
    n_act = int(round(active_frac * nbx * nbx))
    order = np.argsort(-g_b, kind="stable")
    block_active = np.zeros(nbx * nbx, dtype=np.uint8)
    block_active[order[:n_act]] = 1
    mask = _mask_from_blocks((n, n, 1), dim, B, block_active)
    ln_c0 = -2.0 + 1.5 * grf(rs[1], shp, ell)
    ln_c1 = -4.0 + 1.5 * grf(rs[2], shp, ell)
    ln_cc = -6.0 + 0.5 * grf(rs[3], shp, 2 * ell)
    T = _tmap(rs[4], shp, 2 * ell)
    S = np.exp(-1.0 / T)
    vx = 12.0 * grf(rs[5], shp, 2 * ell)
    vy = 12.0 * grf(rs[6], shp, 2 * ell)
    sp = np.sqrt(vx * vx + vy * vy)
    scale = 30.0 / sp[mask].max()
    vx *= scale
    vy *= scale
    lam0 = np.array([500.00, 500.25])
    dv = np.linspace(-60.0, 60.0, n_lam_per_line)
    lam = np.concatenate([l0 * (1.0 + dv / C_KMS) for l0 in lam0])
    vth = 10.0
    chi_star = np.stack([np.exp(ln_c0), np.exp(ln_c1)]) * mask
    eta_star = chi_star * S
    chi_bg = np.exp(ln_cc) * mask
    eta_bg = chi_bg * S
    inv_dld = np.stack([np.full(shp, C_KMS / (l0 * vth)) for l0 in lam0]) * mask
    vel = np.stack([vx, vy]) * mask
    f32 = lambda a, k: a.astype(np.float32).reshape(k, -1)  # noqa: E731
    return dict(
        name="cfg2", dim=dim, n=(n, n, 1), brick=B, n_levels=4, model="lines", profile="gauss",
        lam=lam, lam0=lam0, eta_star=f32(eta_star, 2), chi_star=f32(chi_star, 2),
        damp=np.zeros((2, n * n), np.float32), inv_dld=f32(inv_dld, 2),
        eta_bg=eta_bg.astype(np.float32).reshape(-1), chi_bg=chi_bg.astype(np.float32).reshape(-1),
        vel=f32(vel, 2), dirs=directions_2d(n_dir), block_active=block_active, ds0=1.0, I0=0.0,
        iod_threshold=1e-2, tau_thin=0.25, lam_batch=8, n_v=21, vth=vth,
    )


def make_prominence(seed: int = 6, nx: int = 512, ny: int = 768, B: int = 16, n_lam_per_line: int = 64,
                    n_dir: int = 16, half_width: float = 128.0):
    """2D prominence-like scene for the method matrix: a cool dense sheet (x within
    256 +- half_width, its edges displaced by a Kelvin-Helmholtz-like wave of
    amplitude 24 and wavelength 128 plus a GRF(0, 8, 16) wobble) in a hot corona
    treated as empty (bricks without sheet material have eta = chi = 0, about half
    of them).  Inside: density exp(GRF(0, 0.7, 12)), T = 0.5 + 0.5 Phi(GRF(l=24));
    a thin transition layer (4 voxels) at T = 1.5 and density 0.05.  Two Voigt lines
    (500.0, 500.2 nm; centre opacity 20 n and 1 n per voxel at the reference
    Doppler width 8 km/s; v_D = 8 sqrt(T); damping 10^(-3 + 2 Phi(g))), grey
    continuum 1e-3 n.  Velocity: shear flow v_y = +-20 km/s across the sheet's
    centre line plus a vortical GRF perturbation, rescaled to max |v| = 30 km/s.
    """
    dim = 2
    shp = (ny, nx)
    ss = np.random.SeedSequence(seed)
    rs = [np.random.default_rng(s) for s in ss.spawn(8)]
    yy, xx = np.meshgrid(np.arange(ny) + 0.5, np.arange(nx) + 0.5, indexing="ij")
    wob = 8.0 * grf(rs[0], (ny,), 16.0)
    phase = rs[1].uniform(0, 2 * np.pi)
    edge = half_width + 24.0 * np.sin(2 * np.pi * yy[:, :1] / 128.0 + phase) + wob[:, None]
    dist = np.abs(xx - nx / 2.0) - edge  # < 0 inside the sheet
    inside = dist < 0
    layer = (dist >= 0) & (dist < 4)
    dens = np.where(inside, np.exp(0.7 * grf(rs[2], shp, 12.0)), np.where(layer, 0.05, 0.0))
    T = np.where(inside, 0.5 + 0.5 * ndtr(grf(rs[3], shp, 24.0)), 1.5)
    nbx, nby = nx // B, ny // B
    occ = (dens > 0).reshape(nby, B, nbx, B).any(axis=(1, 3))
    block_active = occ.reshape(-1).astype(np.uint8)  # (by, bx) C order -> bx fastest
    bmask = _mask_from_blocks((nx, ny, 1), dim, B, block_active)
    dens = np.where(bmask & (dens <= 0), 1e-4, dens)
    T = np.where(bmask, T, 1.5)
    S = np.where(bmask, np.exp(-1.0 / T), 0.0)
    vy = 20.0 * np.tanh((xx - nx / 2.0) / 16.0)
    vx = 6.0 * grf(rs[4], shp, 32.0)
    vy = vy + 6.0 * grf(rs[5], shp, 32.0)
    sp = np.sqrt(vx * vx + vy * vy)
    scale = 30.0 / sp[bmask].max()
    vel = np.stack([vx * scale, vy * scale]) * bmask
    lam0 = np.array([500.0, 500.2])
    vD = 8.0 * np.sqrt(T)
    a0 = 10.0 ** (-3.0 + 2.0 * ndtr(grf(rs[6], shp, 16.0)))
    chi_star = np.stack([np.where(bmask, c * dens * math.sqrt(math.pi) * l0 * 8.0 / C_KMS, 0.0)
                         for c, l0 in ((20.0, lam0[0]), (1.0, lam0[1]))])
    inv_dld = np.stack([np.where(bmask, C_KMS / (l0 * vD), 0.0) for l0 in lam0])
    damp = np.stack([np.where(bmask, a0, 0.0)] * 2)
    chi_bg = np.where(bmask, 1e-3 * dens, 0.0)
    dv = np.linspace(-80.0, 80.0, n_lam_per_line)
    lam = np.concatenate([l0 * (1.0 + dv / C_KMS) for l0 in lam0])
    f32 = lambda a, k: a.astype(np.float32).reshape(k, -1)  # noqa: E731
    return dict(
        name="prominence", dim=dim, n=(nx, ny, 1), brick=B, n_levels=4, model="lines", profile="voigt",
        lam=lam, lam0=lam0, eta_star=f32(chi_star * S, 2), chi_star=f32(chi_star, 2), damp=f32(damp, 2),
        inv_dld=f32(inv_dld, 2), eta_bg=(chi_bg * S).astype(np.float32).reshape(-1),
        chi_bg=chi_bg.astype(np.float32).reshape(-1), vel=f32(vel, 2), dirs=directions_2d(n_dir),
        block_active=block_active, ds0=1.0, I0=0.0, iod_threshold=1e-2, tau_thin=0.25, lam_batch=8,
    )


def _loops_density(rng, n, z_top, target_blocks, B, max_loops=400, first=12):
    """Semicircular loop tubes standing on the slab top (z = z_top)."""
    nx = ny = nz = n
    dens = np.zeros((nz, ny, nx), dtype=np.float64)
    temp = np.zeros((nz, ny, nx), dtype=np.float64)
    nbl = n // B
    slab_blocks = int(math.ceil(z_top / B)) * nbl * nbl
    n_loops = 0
    while n_loops < max_loops:
        d = rng.uniform(40.0, 120.0)
        R = 0.5 * d
        r = rng.uniform(3.0, 6.0)
        phi = rng.uniform(0.0, np.pi)
        cx = rng.uniform(R + r, nx - R - r)
        cy = rng.uniform(R + r, ny - R - r)
        tl = rng.uniform(1.2, 2.0)
        ex = np.array([math.cos(phi), math.sin(phi)])
        ext = R + r + 1
        x0, x1 = int(max(0, math.floor(cx - ext))), int(min(nx, math.ceil(cx + ext) + 1))
        y0, y1 = int(max(0, math.floor(cy - ext))), int(min(ny, math.ceil(cy + ext) + 1))
        z0, z1 = z_top, int(min(nz, math.ceil(z_top + R + r) + 1))
        zz, yy, xx = np.meshgrid(np.arange(z0, z1) + 0.5, np.arange(y0, y1) + 0.5,
                                 np.arange(x0, x1) + 0.5, indexing="ij")
        s = (xx - cx) * ex[0] + (yy - cy) * ex[1]
        q = -(xx - cx) * ex[1] + (yy - cy) * ex[0]
        h = zz - z_top
        rho = np.sqrt(s * s + h * h)
        dist = np.sqrt((rho - R) ** 2 + q * q)
        inside = (dist <= r) & (h >= 0)
        val = 0.02 * np.exp(-h / 48.0)
        sub = dens[z0:z1, y0:y1, x0:x1]
        tsub = temp[z0:z1, y0:y1, x0:x1]
        upd = inside & (val > sub)
        sub[upd] = val[upd]
        tsub[upd] = tl
        n_loops += 1
        if n_loops >= first:
            occ = (dens > 0).reshape(nbl, B, nbl, B, nbl, B).any(axis=(1, 3, 5)).sum()
            if occ + slab_blocks >= target_blocks:
                break
    return dens, temp, n_loops


def make_cfg3(seed: int = 3, n: int = 256, B: int = 8, z_slab: int = 48, n_lam_per_line: int = 64,
              n_dir: int = 32, active_target: float = 0.25):
    """3D chromosphere-like slab with loop-shaped filaments and two Voigt lines.

    Slab z < z_slab: density exp(-z/12) exp(GRF(0, 0.5, 8)), T rising 0.6 -> 1.0
    with height; loops add density 0.02 exp(-h/48) at T in [1.2, 2].  Lines at
    500.0 and 500.2 nm, Doppler width 8 sqrt(T) km/s, damping a = 10^(-3 + 2 Phi(g))
    in [1e-3, 1e-1]; line-centre opacity chi*_l H(a,0)/(sqrt(pi) dlD_ref) set to
    {50, 2} x density at the reference width 8 km/s; grey continuum 1e-3 density.
    Velocity: three GRF(0, 10 km/s, 32) components, rescaled to max |v| = 30 km/s.
    """
    dim = 3
    shp = (n, n, n)  # (z, y, x)
    ss = np.random.SeedSequence(seed)
    rs = [np.random.default_rng(s) for s in ss.spawn(7)]
    nbl = n // B
    target = int(round(active_target * nbl ** 3))
    dens_l, t_l, n_loops = _loops_density(rs[0], n, z_slab, target, B)
    g8 = grf(rs[1], (z_slab, n, n), 8.0)
    z = np.arange(z_slab, dtype=np.float64)[:, None, None] + 0.5
    dens = dens_l
    dens[:z_slab] = np.exp(-z / 12.0) * np.exp(0.5 * g8)
    T = t_l
    T[:z_slab] = 0.6 + 0.4 * (z / z_slab) * np.ones((1, n, n))
    mask = dens > 0
    occ = mask.reshape(nbl, B, nbl, B, nbl, B).any(axis=(1, 3, 5))
    block_active = occ.reshape(-1).astype(np.uint8)  # (bz, by, bx) C order -> bx fastest
    bmask = _mask_from_blocks((n, n, n), dim, B, block_active)
    T = np.where(bmask & ~mask, 1.0, T)
    dens = np.where(bmask & ~mask, 1e-6, dens)  # keep every voxel of an active brick positive
    S = np.where(bmask, np.exp(-1.0 / np.maximum(T, 1e-3)), 0.0)
    vc = [10.0 * grf(rs[2 + i], shp, 32.0) for i in range(3)]
    sp = np.sqrt(vc[0] ** 2 + vc[1] ** 2 + vc[2] ** 2)
    scale = 30.0 / sp[bmask].max()
    vel = np.stack([v * scale for v in vc]) * bmask
    lam0 = np.array([500.0, 500.2])
    vD = 8.0 * np.sqrt(np.maximum(T, 1e-3))
    ga = grf(rs[5], shp, 16.0)
    a0 = 10.0 ** (-3.0 + 2.0 * ndtr(ga))
    chi_star, inv_dld = [], []
    for l, l0 in enumerate(lam0):
        dld_ref = l0 * 8.0 / C_KMS
        chi_star.append(np.where(bmask, (50.0 if l == 0 else 2.0) * dens * math.sqrt(math.pi) * dld_ref, 0.0))
        inv_dld.append(np.where(bmask, C_KMS / (l0 * vD), 0.0))
    chi_star = np.stack(chi_star)
    inv_dld = np.stack(inv_dld)
    eta_star = chi_star * S
    damp = np.stack([np.where(bmask, a0, 0.0)] * 2)
    chi_bg = np.where(bmask, 1e-3 * dens, 0.0)
    eta_bg = chi_bg * S
    dv = np.linspace(-80.0, 80.0, n_lam_per_line)
    lam = np.concatenate([l0 * (1.0 + dv / C_KMS) for l0 in lam0])
    f32 = lambda a, k: a.astype(np.float32).reshape(k, -1)  # noqa: E731
    return dict(
        name="cfg3", dim=dim, n=(n, n, n), brick=B, n_levels=4, model="lines", profile="voigt",
        lam=lam, lam0=lam0, eta_star=f32(eta_star, 2), chi_star=f32(chi_star, 2),
        damp=f32(damp, 2), inv_dld=f32(inv_dld, 2),
        eta_bg=eta_bg.astype(np.float32).reshape(-1), chi_bg=chi_bg.astype(np.float32).reshape(-1),
        vel=f32(vel, 3), dirs=directions_fibonacci(n_dir), block_active=block_active,
        ds0=1.0, I0=0.0, iod_threshold=1e-2, tau_thin=0.25, lam_batch=8, n_loops=n_loops,
    )


def cfg4_specs(seed: int = 4000, n_scenes: int = 48):
    """Per-scene shapes of the uneven batch (seeded)."""
    specs = []
    for i in range(n_scenes):
        rng = np.random.default_rng(np.random.SeedSequence(seed + i))
        if i < n_scenes // 2:
            k = int(rng.integers(0, 5))
            N, dim, B = 64 * 2 ** k, 2, 16
            L = int(rng.integers(2, 6))
        else:
            N = int(rng.choice([64, 96, 128, 160, 192]))
            dim, B = 3, 8
            L = int(rng.integers(2, 5))
        n_dir = int(rng.choice([16, 32, 64]))
        n_lam = int(rng.choice([64, 128, 192, 256]))
        specs.append(dict(index=i, seed=seed + i, N=N, dim=dim, brick=B, n_levels=L,
                          n_dir=n_dir, n_lam=n_lam))
    return specs


def make_cfg4_scene(spec, empty_frac: float = 0.3):
    """One scene of the uneven batch: cfg1 recipe (ell = N/10) as a static line +
    continuum in the line-parameter form (zero velocity), evaluated per batch."""
    dim, N, B = spec["dim"], spec["N"], spec["brick"]
    shp = (N,) * dim
    ss = np.random.SeedSequence(spec["seed"])
    rs = [np.random.default_rng(s) for s in ss.spawn(4)]
    ell = N / 10.0
    ln_chi = -2.0 + 1.5 * grf(rs[0], shp, ell)
    ln_cc = -6.0 + 0.5 * grf(rs[1], shp, 2 * ell)
    T = _tmap(rs[2], shp, 2 * ell)
    S = np.exp(-1.0 / T)
    nb = (N // B) ** dim
    n_empty = int(round(empty_frac * nb))
    block_active = np.ones(nb, dtype=np.uint8)
    block_active[rs[3].choice(nb, size=n_empty, replace=False)] = 0
    n3 = (N, N, N if dim == 3 else 1)
    mask = _mask_from_blocks(n3, dim, B, block_active)
    lam0 = np.array([500.0])
    vth = 10.0
    dv = np.linspace(-40.0, 40.0, spec["n_lam"])
    lam = lam0[0] * (1.0 + dv / C_KMS)
    chi_star = (np.exp(ln_chi) * mask)[None]
    eta_star = chi_star * S
    chi_bg = np.exp(ln_cc) * mask
    eta_bg = chi_bg * S
    inv_dld = (np.full(shp, C_KMS / (lam0[0] * vth)) * mask)[None]
    vel = np.zeros((dim,) + shp)
    f32 = lambda a, k: a.astype(np.float32).reshape(k, -1)  # noqa: E731
    dirs = directions_2d(spec["n_dir"]) if dim == 2 else directions_fibonacci(spec["n_dir"])
    return dict(
        name="cfg4_%02d" % spec["index"], dim=dim, n=n3, brick=B, n_levels=spec["n_levels"],
        model="lines", profile="gauss", lam=lam, lam0=lam0, eta_star=f32(eta_star, 1),
        chi_star=f32(chi_star, 1), damp=np.zeros((1, int(np.prod(shp))), np.float32),
        inv_dld=f32(inv_dld, 1), eta_bg=eta_bg.astype(np.float32).reshape(-1),
        chi_bg=chi_bg.astype(np.float32).reshape(-1), vel=f32(vel, dim), dirs=dirs,
        block_active=block_active, ds0=1.0, I0=0.0, iod_threshold=1e-2, tau_thin=0.25,
        lam_batch=8,
    )
