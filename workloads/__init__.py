"""Seeded synthetic inputs shared by the oracle and the GPU path.

This module only draws and lays out inputs (densities, temperature, solid
mask, wall temperature, model constants). It holds none of the lattice
Boltzmann arithmetic; both the oracle and the GPU library receive the same
arrays and compute everything else on their own.

The paper prepares its emulsions from droplet layouts (Sec. 3.2.1, the
preparation table of Appendix A) and studies convection between a hot bottom
and a cold top wall (Sec. 3.2.3) with flat or rough walls (Sec. 4). No public
dataset is involved; the layouts below stand in for the paper's prepared
emulsions at the sizes the benchmarks need:

=====  ===========  ======================================================
name   lattice      content
=====  ===========  ======================================================
small  128 x 64     6 discs R=8 (rejection sampled), linear T, FP64 parity
mid    1024 x 512   42 x 21 discs R=10 on a jittered grid, density and T noise
large  4096 x 2048  167 x 84 discs R=10 above bottom posts 8x8, gaps 16..64
crop   512 x 256    the 'large' recipe on a smaller lattice (precision study)
=====  ===========  ======================================================

Droplets are sharp discs: component A at ``rho_in`` inside and ``rho_out``
outside, component B the other way round. Temperature is the conduction
profile between the walls (bottom wall at 1, top at 0, wall planes half a
cell outside the first and last rows) plus optional uniform noise.
"""
from __future__ import annotations

import numpy as np

# Model constants of the paper's preparation/convection tables (Appendix A),
# with the repulsive couplings taken positive as the text of Sec. 2.1 states.
BASE_PARAMS = dict(
    tau=1.0,
    tau_g=1.0,
    rho0=0.83,
    g12=0.405,
    g_a=(-9.0, -8.0),
    g_r=(8.1, 7.1),
    alpha_g=1.0e-4,
    t_top=0.0,
    rho_wall=(0.612, 0.612),
    dt_nominal=1.0,
)

RHO_IN, RHO_OUT = 1.36, 0.08


def _rng(seed: int) -> np.random.Generator:
    return np.random.Generator(np.random.PCG64(seed))


def conduction_profile(lx: int, ly: int, t_bottom: float = 1.0, t_top: float = 0.0) -> np.ndarray:
    """Linear profile with the wall planes at y = -1/2 and y = ly - 1/2."""
    y = (np.arange(ly) + 0.5) / ly
    return np.repeat((t_bottom + (t_top - t_bottom) * y)[:, None], lx, axis=1)


def paint_discs(lx: int, ly: int, centres, radius: float):
    """Boolean mask of the union of discs (periodic in x)."""
    inside = np.zeros((ly, lx), bool)
    r = int(np.ceil(radius))
    ys = np.arange(ly)
    for cx, cy in centres:
        y0, y1 = max(int(np.floor(cy - r)), 0), min(int(np.ceil(cy + r)) + 1, ly)
        xs = np.arange(int(np.floor(cx - r)), int(np.ceil(cx + r)) + 1)
        dx = xs - cx
        dy = ys[y0:y1] - cy
        hit = dx[None, :] ** 2 + dy[:, None] ** 2 <= radius * radius
        inside[y0:y1, xs % lx] |= hit
    return inside


def jittered_grid(rng, nx: int, ny: int, x_span, y_span, jitter: float):
    """nx*ny centres on a regular grid over the spans, jittered uniformly."""
    (x0, x1), (y0, y1) = x_span, y_span
    sx, sy = (x1 - x0) / nx, (y1 - y0) / ny
    gx = x0 + (np.arange(nx) + 0.5) * sx
    gy = y0 + (np.arange(ny) + 0.5) * sy
    cx, cy = np.meshgrid(gx, gy)
    cx = cx.ravel() + rng.uniform(-jitter, jitter, cx.size)
    cy = cy.ravel() + rng.uniform(-jitter, jitter, cy.size)
    return np.stack([cx, cy], axis=1)


def bottom_posts(rng, lx: int, ly: int, height: int = 8, width: int = 8,
                 gap=(16, 64)) -> np.ndarray:
    """Solid mask (uint8, 1 = solid held at the bottom temperature) with
    rectangular posts on the bottom wall, separated by seeded integer gaps
    drawn from ``gap`` (inclusive) and placed from a seeded offset; the last
    post is dropped if the periodic wrap would leave a gap below gap[0]."""
    solid = np.zeros((ly, lx), np.uint8)
    x = int(rng.integers(0, gap[1]))
    first = x
    while True:
        if x + width + gap[0] > first + lx:
            break
        solid[:height, np.arange(x, x + width) % lx] = 1
        x += width + int(rng.integers(gap[0], gap[1] + 1))
    return solid


def _emulsion(lx, ly, seed, n_x, n_y, radius, noise_rho, noise_t, posts, jitter=2.0):
    rng = _rng(seed)
    solid = bottom_posts(rng, lx, ly) if posts else None
    y_lo = 8 if posts else 0
    centres = jittered_grid(rng, n_x, n_y, (0, lx), (y_lo, ly), jitter)
    inside = paint_discs(lx, ly, centres, radius)
    rho_a = np.where(inside, RHO_IN, RHO_OUT)
    rho_b = np.where(inside, RHO_OUT, RHO_IN)
    if noise_rho:
        rho_a = rho_a + rng.uniform(-noise_rho, noise_rho, rho_a.shape)
        rho_b = rho_b + rng.uniform(-noise_rho, noise_rho, rho_b.shape)
    temp = conduction_profile(lx, ly)
    if noise_t:
        temp = temp + rng.uniform(-noise_t, noise_t, temp.shape)
    return dict(rho_a=rho_a, rho_b=rho_b, temp=temp, solid=solid,
                t_bottom=np.ones(lx), n_droplets=len(centres),
                area_fraction=float(inside.mean()))


def small(seed: int = 1, steps: int = 200, alpha_g: float = 1e-4) -> dict:
    """128 x 64, six discs R=8: centre distance >= 2R+4, wall clearance
    >= R+3, rejection sampled."""
    lx, ly, radius = 128, 64, 8.0
    rng = _rng(seed)
    centres = []
    while len(centres) < 6:
        c = np.array([rng.uniform(0, lx), rng.uniform(radius + 3, ly - radius - 3)])
        ok = True
        for d in centres:
            dx = abs(c[0] - d[0])
            dx = min(dx, lx - dx)
            if dx * dx + (c[1] - d[1]) ** 2 < (2 * radius + 4) ** 2:
                ok = False
                break
        if ok:
            centres.append(c)
    inside = paint_discs(lx, ly, centres, radius)
    params = dict(BASE_PARAMS, alpha_g=alpha_g)
    return dict(name="small-128x64", lx=lx, ly=ly, seed=seed, steps=steps, params=params,
                rho_a=np.where(inside, RHO_IN, RHO_OUT), rho_b=np.where(inside, RHO_OUT, RHO_IN),
                temp=conduction_profile(lx, ly), solid=None, t_bottom=np.ones(lx),
                n_droplets=6, area_fraction=float(inside.mean()))


def mid(seed: int = 2, steps: int = 2000) -> dict:
    """1024 x 512, 42 x 21 = 882 discs R=10, density noise U(-0.01, 0.01),
    temperature noise U(-1e-3, 1e-3), flat walls."""
    d = _emulsion(1024, 512, seed, 42, 21, 10.0, 0.01, 1e-3, posts=False)
    return dict(d, name="mid-1024x512", lx=1024, ly=512, seed=seed, steps=steps,
                params=dict(BASE_PARAMS))


def large(seed: int = 3, steps: int = 1000) -> dict:
    """4096 x 2048, 167 x 84 = 14028 discs R=10 above seeded 8 x 8 bottom
    posts with gaps 16..64, noise as in ``mid``."""
    d = _emulsion(4096, 2048, seed, 167, 84, 10.0, 0.01, 1e-3, posts=True)
    return dict(d, name="large-4096x2048", lx=4096, ly=2048, seed=seed, steps=steps,
                params=dict(BASE_PARAMS))


def large_flat(seed: int = 3, steps: int = 500) -> dict:
    """4096 x 2048 with the ``large`` recipe but flat walls (no posts): the
    full-size lattice for the adjoint, which takes flat walls only."""
    d = _emulsion(4096, 2048, seed, 167, 84, 10.0, 0.01, 1e-3, posts=False)
    return dict(d, name="large-flat-4096x2048", lx=4096, ly=2048, seed=seed, steps=steps,
                params=dict(BASE_PARAMS))


def crop(seed: int = 4, steps: int = 5000) -> dict:
    """512 x 256 lattice built with the 'large' recipe (21 x 10 discs)."""
    d = _emulsion(512, 256, seed, 21, 10, 10.0, 0.01, 1e-3, posts=True)
    return dict(d, name="crop-512x256", lx=512, ly=256, seed=seed, steps=steps,
                params=dict(BASE_PARAMS))


def adjoint_strip(seed: int = 2, steps: int = 500) -> dict:
    """1024 x 64 strip with the ``mid`` recipe (42 x 2 discs R=10, same
    noise): the width of ``mid`` with the top wall inside the bottom wall's
    domain of dependence over a few hundred steps."""
    d = _emulsion(1024, 64, seed, 42, 2, 10.0, 0.01, 1e-3, posts=False)
    return dict(d, name="strip-1024x64", lx=1024, ly=64, seed=seed, steps=steps,
                params=dict(BASE_PARAMS))


def bottom_temperature_noise(lx: int, seed: int = 5, amplitude: float = 1e-2) -> np.ndarray:
    """Bottom-wall temperature 1 + U(-amplitude, amplitude) per column."""
    return 1.0 + _rng(seed).uniform(-amplitude, amplitude, lx)


def two_layer(lx: int = 128, ly: int = 2, rho_max: float = 1.4, rho_min: float = 0.1,
              rich_columns: int = 65) -> dict:
    """Two-layer start of the phase-separation experiment (Appendix B):
    columns [0, rich_columns) rich in component A, the rest rich in B."""
    rich = (np.arange(lx) < rich_columns)[None, :].repeat(ly, axis=0)
    return dict(rho_a=np.where(rich, rho_max, rho_min), rho_b=np.where(rich, rho_min, rho_max),
                temp=np.zeros((ly, lx)))


def single_droplet(lx: int, ly: int, radius: float) -> dict:
    """One disc at the box centre (for the Laplace test)."""
    inside = paint_discs(lx, ly, [((lx - 1) / 2.0, (ly - 1) / 2.0)], radius)
    return dict(rho_a=np.where(inside, RHO_IN, RHO_OUT), rho_b=np.where(inside, RHO_OUT, RHO_IN),
                temp=np.zeros((ly, lx)))


CONFIGS = {"small": small, "mid": mid, "large": large, "large-flat": large_flat, "crop": crop,
           "strip": adjoint_strip}
