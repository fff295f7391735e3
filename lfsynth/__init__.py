"""Seeded synthetic light fields shaped like the paper's workloads.

This module is the only code shared by the oracle side and the GPU side.  It
renders inputs (views, a hypothesis list, ground-truth disparity) and holds
the workload definitions (shapes and method parameters); it contains none of
the depth method's arithmetic (no Census, no matching cost, no SGM).

Geometry follows the two-plane light field of the paper's Sec. 3.1: a scene
point at reference pixel (u, v) with disparity d appears in view (s, t) at
(u + (s_hat - s) d, v + (t_hat - t) d), Eq. (1).  A scene is a list of planes
d_j(u, v) = a + b (u - uc) + c (v - vc) with a support region in reference
coordinates (plane 0 covers everything); at each view pixel the visible plane
is the one with the largest d among those whose support contains the
back-projected point.  Textures are rasters on the integer lattice of
reference coordinates, sampled bilinearly.

The paper evaluates on the 4D Light Field Benchmark (9x9 views of 512x512,
Sec. 4.1), EPFL/Lytro and Middlebury scenes; none of them is available here,
so these seeded scenes of the same shapes stand in for them.
"""
from __future__ import annotations

import dataclasses
import numpy as np

__all__ = [
    "Plane", "Scene", "LightField", "perlin2", "fbm", "render", "hypotheses",
    "two_plane_scene", "slanted_scene", "workload", "WORKLOADS",
]


# ----------------------------------------------------------------------------
# Perlin gradient noise, written from Perlin's published "improved noise"
# construction (quintic fade 6t^5 - 15t^4 + 10t^3, hashed lattice gradients).
# ----------------------------------------------------------------------------
_GRADS = np.array([[1, 1], [-1, 1], [1, -1], [-1, -1],
                   [1, 0], [-1, 0], [0, 1], [0, -1]], dtype=np.float64)
_GX, _GY = np.ascontiguousarray(_GRADS[:, 0]), np.ascontiguousarray(_GRADS[:, 1])


def _fade(t):
    return t * t * t * (t * (t * 6.0 - 15.0) + 10.0)


def perlin2(x, y, perm):
    """2-D gradient noise at float arrays x, y with a doubled permutation table."""
    xi = np.floor(x)
    yi = np.floor(y)
    xf = x - xi
    yf = y - yi
    X = xi.astype(np.int64) & 255
    Y = yi.astype(np.int64) & 255
    u = _fade(xf)
    v = _fade(yf)

    def grad(h, dx, dy):
        i = h & 7
        return _GX[i] * dx + _GY[i] * dy

    pX, pX1 = perm[X], perm[X + 1]
    aa = perm[pX + Y]
    ab = perm[pX + Y + 1]
    ba = perm[pX1 + Y]
    bb = perm[pX1 + Y + 1]
    g_aa = grad(aa, xf, yf)
    g_ab = grad(ab, xf, yf - 1)
    x1 = g_aa + u * (grad(ba, xf - 1, yf) - g_aa)
    x2 = g_ab + u * (grad(bb, xf - 1, yf - 1) - g_ab)
    return x1 + v * (x2 - x1)


def fbm(x, y, perm, octaves=4):
    """Fractal sum of `octaves` Perlin octaves, normalised to roughly [-1, 1]."""
    acc = np.zeros_like(x, dtype=np.float64)
    amp, freq, norm = 1.0, 1.0, 0.0
    for _ in range(octaves):
        acc += amp * perlin2(x * freq, y * freq, perm)
        norm += amp
        amp *= 0.5
        freq *= 2.0
    return acc / norm


# ----------------------------------------------------------------------------
# Scene description
# ----------------------------------------------------------------------------
@dataclasses.dataclass
class Plane:
    a: float                   # disparity at (uc, vc)
    b: float                   # d/du
    c: float                   # d/dv
    uc: float
    vc: float
    ax: float = np.inf         # ellipse semi-axes of the support (inf: everywhere)
    ay: float = np.inf
    square: bool = False       # support is the axis-aligned box |u-uc|<ax, |v-vc|<ay
    texture: np.ndarray = None  # float64 raster, index [v + margin, u + margin]
    margin: int = 0


@dataclasses.dataclass
class Scene:
    H: int
    W: int
    planes: list


@dataclasses.dataclass
class LightField:
    views: np.ndarray          # [T][S][H][W] or [T][S][C][H][W], uint8 or float32
    hyp: np.ndarray            # [N] float32, strictly increasing
    gt: np.ndarray             # [H][W] float32 ground-truth disparity (reference view)
    params: dict               # method parameters for this workload
    name: str = ""

    @property
    def S(self):
        return self.views.shape[1]

    @property
    def T(self):
        return self.views.shape[0]

    @property
    def C(self):
        return 1 if self.views.ndim == 4 else self.views.shape[2]

    @property
    def H(self):
        return self.views.shape[-2]

    @property
    def W(self):
        return self.views.shape[-1]

    @property
    def N(self):
        return self.hyp.shape[0]


def hypotheses(d_min, d_max, N):
    """d_k = d_min + k (d_max - d_min) / (N - 1), computed in double, stored as float32."""
    k = np.arange(N, dtype=np.float64)
    return (d_min + k * (d_max - d_min) / (N - 1)).astype(np.float32)


def _bilinear(raster, x, y):
    """Bilinear lookup of a 2-D raster at float coordinates (clamped to the raster)."""
    h, w = raster.shape
    x = np.clip(x, 0.0, w - 1.000001)
    y = np.clip(y, 0.0, h - 1.000001)
    x0 = np.floor(x).astype(np.int64)
    y0 = np.floor(y).astype(np.int64)
    fx = x - x0
    fy = y - y0
    a = raster[y0, x0]
    b = raster[y0, x0 + 1]
    c = raster[y0 + 1, x0]
    e = raster[y0 + 1, x0 + 1]
    top = a + fx * (b - a)
    bot = c + fx * (e - c)
    return top + fy * (bot - top)


def render(scene: Scene, S: int, T: int, dtype=np.float32, noise_sigma=0.0, rng=None):
    """Render all S x T views of a plane scene; returns (views[T][S][H][W], gt[H][W]),
    or views[T][S][C][H][W] when the textures have C channels ([C][rows][cols]).

    uint8 output takes texture values in 0..255 units (rounded half to even); float32
    output takes them in [0, 1].
    """
    tex0 = scene.planes[0].texture
    if tex0.ndim == 3:                           # colour: one pass per channel plane
        planes = []
        gt = None
        for c in range(tex0.shape[0]):
            sc = Scene(scene.H, scene.W, [dataclasses.replace(pl, texture=pl.texture[c])
                                          for pl in scene.planes])
            v, gt = render(sc, S, T, dtype, noise_sigma, rng)
            planes.append(v)
        return np.ascontiguousarray(np.stack(planes, axis=2)), gt
    H, W = scene.H, scene.W
    sh, th = (S - 1) / 2.0, (T - 1) / 2.0
    yy, xx = np.meshgrid(np.arange(H, dtype=np.float64), np.arange(W, dtype=np.float64),
                         indexing="ij")
    views = np.empty((T, S, H, W), dtype=dtype)
    # the noise of every view is drawn first, in view order, so that the views can
    # be rendered in any order with the same values
    noise = {}
    if noise_sigma > 0:
        for t in range(T):
            for s in range(S):
                noise[t, s] = rng.normal(0.0, noise_sigma, size=(H, W))

    def one_view(ts):
        t, s = ts
        cs, ct = sh - s, th - t
        best_d = np.full((H, W), -np.inf)
        best_j = np.full((H, W), -1, dtype=np.int64)
        best_u = np.zeros((H, W))
        best_v = np.zeros((H, W))
        for j, pl in enumerate(scene.planes):
            # x = u + cs d(u,v), y = v + ct d(u,v) with d linear in (u, v)
            k0 = pl.a - pl.b * pl.uc - pl.c * pl.vc
            m00, m01 = 1.0 + cs * pl.b, cs * pl.c
            m10, m11 = ct * pl.b, 1.0 + ct * pl.c
            det = m00 * m11 - m01 * m10
            rx = xx - cs * k0
            ry = yy - ct * k0
            u = (m11 * rx - m01 * ry) / det
            v = (m00 * ry - m10 * rx) / det
            d = pl.a + pl.b * (u - pl.uc) + pl.c * (v - pl.vc)
            if np.isinf(pl.ax):
                inside = np.ones((H, W), dtype=bool)
            elif pl.square:
                inside = (np.abs(u - pl.uc) < pl.ax) & (np.abs(v - pl.vc) < pl.ay)
            else:
                inside = ((u - pl.uc) / pl.ax) ** 2 + ((v - pl.vc) / pl.ay) ** 2 <= 1.0
            take = inside & (d > best_d)
            best_d = np.where(take, d, best_d)
            best_j = np.where(take, j, best_j)
            best_u = np.where(take, u, best_u)
            best_v = np.where(take, v, best_v)
        img = np.zeros((H, W))
        for j, pl in enumerate(scene.planes):
            sel = best_j == j
            if not sel.any():
                continue
            img[sel] = _bilinear(pl.texture, best_u[sel] + pl.margin, best_v[sel] + pl.margin)
        if noise_sigma > 0:
            img = img + noise[t, s]
        if np.dtype(dtype) == np.uint8:
            views[t, s] = np.clip(np.rint(img), 0, 255).astype(np.uint8)
        else:
            views[t, s] = np.clip(img, 0.0, 1.0).astype(np.float32)
        return best_d.astype(np.float32)

    depth = _parallel_map(one_view, [(t, s) for t in range(T) for s in range(S)])
    gt = depth[((T - 1) // 2) * S + (S - 1) // 2]
    return views, gt


# ----------------------------------------------------------------------------
# Scene families
# ----------------------------------------------------------------------------
def _noise_lattice(rng, H, W, margin):
    """i.i.d. uniform U{0..255} lattice (float64), the texture of the small plain workload."""
    return rng.integers(0, 256, size=(H + 2 * margin + 2, W + 2 * margin + 2)).astype(np.float64)


def two_plane_scene(seed, H=96, W=96, d_back=-1.25, d_front=0.75, S=5, T=5):
    """Background fronto-parallel plane plus a centred square foreground plane."""
    rng = np.random.default_rng(seed)
    margin = int(np.ceil(max(S, T) / 2.0 * max(abs(d_back), abs(d_front)))) + 3
    back = Plane(a=d_back, b=0.0, c=0.0, uc=W / 2.0, vc=H / 2.0,
                 texture=_noise_lattice(rng, H, W, margin), margin=margin)
    front = Plane(a=d_front, b=0.0, c=0.0, uc=W / 2.0, vc=H / 2.0, ax=W / 4.0, ay=H / 4.0,
                  square=True, texture=_noise_lattice(rng, H, W, margin), margin=margin)
    return Scene(H, W, [back, front])


def _draw_perlin_texture(rng, H, W, margin):
    """The random draws of one Perlin+noise texture, in their fixed order; the
    texture itself is computed later by _perlin_from_draws (so that several can be
    computed at once without changing any value)."""
    perm = rng.permutation(256)
    perm = np.concatenate([perm, perm]).astype(np.int64)
    sigma = rng.uniform(16.0, 64.0)
    hh, ww = H + 2 * margin + 2, W + 2 * margin + 2
    ox, oy = rng.uniform(0, 256, size=2)
    noise = rng.uniform(0.0, 1.0, size=(hh, ww))
    return (perm, sigma, ox, oy, noise)


def _perlin_from_draws(draws):
    perm, sigma, ox, oy, noise = draws
    hh, ww = noise.shape
    yy, xx = np.meshgrid(np.arange(hh, dtype=np.float64), np.arange(ww, dtype=np.float64),
                         indexing="ij")
    f = fbm(xx / sigma + ox, yy / sigma + oy, perm, octaves=4)
    return np.clip(0.5 + 0.35 * f + 0.15 * (noise - 0.5), 0.0, 1.0)


def _parallel_map(fn, items):
    """map() over a thread pool (numpy releases the GIL in the array work); the
    results do not depend on the schedule."""
    import concurrent.futures as cf
    import os
    items = list(items)
    if len(items) <= 1:
        return [fn(x) for x in items]
    with cf.ThreadPoolExecutor(max_workers=min(len(items), os.cpu_count() or 1, 16)) as ex:
        return list(ex.map(fn, items))


def _perlin_texture(rng, H, W, margin):
    return _perlin_from_draws(_draw_perlin_texture(rng, H, W, margin))


def slanted_scene(seed, H, W, d_min, d_max, n_planes=12, S=9, T=9, channels=1):
    """Background plane plus (n_planes - 1) slanted elliptical planes, Perlin+noise textures
    (channels = 3: an independent texture per colour channel)."""
    rng = np.random.default_rng(seed)

    # each texture's random draws are taken here in order; the textures are computed
    # together at the end
    def texture():
        return [_draw_perlin_texture(rng, H, W, margin) for _ in range(channels)]

    span = d_max - d_min
    margin = int(np.ceil(max(S, T) / 2.0 * max(abs(d_min), abs(d_max)))) + 3
    planes = []
    # background: the far end of the range, gently slanted
    a0 = d_min + span * rng.uniform(0.1, 0.25)
    room = min(a0 - d_min, d_max - a0)
    b0, c0 = rng.uniform(-1, 1, size=2) * room / (W + H)
    planes.append(Plane(a=a0, b=b0, c=c0, uc=W / 2.0, vc=H / 2.0,
                        texture=texture(), margin=margin))
    scale = min(H, W) / 512.0
    for _ in range(n_planes - 1):
        uc, vc = rng.uniform(0, W), rng.uniform(0, H)
        ax, ay = rng.uniform(20.0, 100.0, size=2) * max(scale, 0.25)
        a = rng.uniform(d_min, d_max)
        room = max(min(a - d_min, d_max - a), 0.0)
        b, c = rng.uniform(-1, 1, size=2) * 0.02 * span / 8.0
        reach = abs(b) * ax + abs(c) * ay
        if reach > room:
            f = room / reach if reach > 0 else 0.0
            b, c = b * f, c * f
        planes.append(Plane(a=a, b=b, c=c, uc=uc, vc=vc, ax=ax, ay=ay,
                            texture=texture(), margin=margin))
    flat = [d for pl in planes for d in pl.texture]
    tex = _parallel_map(_perlin_from_draws, flat)
    for j, pl in enumerate(planes):
        t = tex[j * channels:(j + 1) * channels]
        pl.texture = t[0] if channels == 1 else np.stack(t)
    return Scene(H, W, planes)


# ----------------------------------------------------------------------------
# Workloads (shapes, seeds and the method parameters used for each)
# ----------------------------------------------------------------------------
def _params(census=(5, 5), p_init=(10, 120), p_final=(10, 120), lam=2, phi=3, fill=2,
            edge_tau=float("inf"), alpha=1.0, sum_bits=16, npaths=8, cost_kind=0, median=3):
    return dict(win_h=census[0], win_w=census[1], P1_init=p_init[0], P2_init=p_init[1],
                P1_final=p_final[0], P2_final=p_final[1], npaths=npaths, lam=lam, phi=phi,
                fill_passes=fill, edge_tau=edge_tau, alpha=alpha, sum_bits=sum_bits,
                cost_kind=cost_kind, median=median)


def checkerboard_census_offsets(win_h, win_w):
    """A sparse Census window (Sec. 3.2) as a neighbour list: the pixels of the
    win_h x win_w window whose offsets (dy, dx) have an even sum, the centre left
    out, in row-major order (24 comparisons for 7 x 7).  The paper's own sparse
    7 x 7 pattern comes from another publication and is not reproduced here; this
    one is a stand-in of the same size class."""
    return [(i, j) for i in range(-(win_h // 2), win_h // 2 + 1)
            for j in range(-(win_w // 2), win_w // 2 + 1)
            if (i + j) % 2 == 0 and (i, j) != (0, 0)]


def _small_plain(seed=1, H=96, W=96, S=5, T=5, N=32):
    scene = two_plane_scene(seed, H, W, S=S, T=T)
    views, gt = render(scene, S, T, dtype=np.uint8)
    return LightField(views, hypotheses(-2.0, 2.0, N), gt, _params(), name="lf5x5_96_u8")


def _paper_shape(seed=2, H=512, W=512, S=9, T=9, N=100, d_min=-4.0, d_max=4.0, noise=0.0,
                 channels=1):
    scene = slanted_scene(seed, H, W, d_min, d_max, S=S, T=T, channels=channels)
    rng = np.random.default_rng(seed + 7919)
    views, gt = render(scene, S, T, dtype=np.float32, noise_sigma=noise, rng=rng)
    p = _params(census=(7, 9), p_init=(21, 45), p_final=(17, 35), lam=3, phi=3, fill=2,
                edge_tau=128.0, alpha=255.0, sum_bits=32)
    return LightField(views, hypotheses(d_min, d_max, N), gt, p,
                      name=f"lf{S}x{T}_{H}x{W}_f32_N{N}")


def _moving_stage(seed, H=1080, W=1920, S=11, N=96):
    scene = slanted_scene(seed, H, W, 0.0, 24.0, S=S, T=1)
    views, gt = render(scene, S, 1, dtype=np.float32)
    views = np.clip(np.rint(views.astype(np.float64) * 255.0), 0, 255).astype(np.uint8)
    p = _params(census=(7, 9), p_init=(21, 45), p_final=(17, 35), lam=3, phi=3, fill=2,
                edge_tau=128.0, alpha=1.0, sum_bits=32)
    return LightField(views, hypotheses(0.0, 24.0, N), gt, p, name=f"lf{S}x1_{H}x{W}_u8_N{N}")


def workload(name: str, seed=None, **kw) -> LightField:
    """Build one named workload.

    small      5x5 views of 96x96 u8, two fronto-parallel planes (d = -1.25, +0.75),
               uniform-noise texture, N = 32 over [-2, 2], 5x5 Census, P1/P2 = 10/120.
    paper      9x9 views of 512x512 f32 in [0, 1], 12 slanted Perlin+noise planes,
               N = 100 over [-4, 4], 7x9 Census, lambda = 3, P1/P2 21/45 and 17/35.
    paper_s    same family at a reduced size (kw: H, W, S, T, N) for parity tests.
    plenoptic  15x15 views of 625x434 f32, d in [-1.5, 1.5], N = 64, noise 0.01.
    stage      1x11 views of 1920x1080 u8 (moving stage), d in [0, 24], N = 96.
    """
    if name == "small":
        return _small_plain(seed if seed is not None else 1, **kw)
    if name == "paper":
        return _paper_shape(seed if seed is not None else 2, **kw)
    if name == "paper_s":
        return _paper_shape(seed if seed is not None else 2, **kw)
    if name == "plenoptic":
        return _paper_shape(seed if seed is not None else 4001, H=434, W=625, S=15, T=15,
                            N=64, d_min=-1.5, d_max=1.5, noise=0.01)
    if name == "stage":
        return _moving_stage(seed if seed is not None else 4003, **kw)
    raise KeyError(name)


WORKLOADS = ("small", "paper", "paper_s", "plenoptic", "stage")
