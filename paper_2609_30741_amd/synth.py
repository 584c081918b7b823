"""Seeded synthetic inputs: 2DGS surfel scenes, pinhole stereo rigs and
stage-level test images.

This module holds input generation only; none of the rendering,
reprojection or hole-classification arithmetic lives here.  Both the HIP
path and the CPU oracle consume exactly the bytes produced here (fp32
arrays), so the two sides always see identical inputs.

Conventions (the paper's pinhole model, Sec. 3.4 Eq. 3-5):
  * camera frame is x right, y down, z forward; depth is z along the
    optical axis;
  * a camera pose (R, t) maps camera to world: X_w = R X_c + t, so the
    world-to-camera map is X_c = R^T (X_w - t);
  * pixel (i, j) has its centre at continuous coordinates (i, j), and the
    principal point is the image centre ((W-1)/2, (H-1)/2);
  * the stereo rig keeps the orientation and offsets the affiliated eye
    along the dominant camera's x axis (Sec. 4.2).

Scene layout (structure of arrays, all fp32, activated values):
  pos[3][n], quat[4][n] (w, x, y, z; unit), scale[2][n] (s_u, s_v > 0),
  opacity[n] in (0, 1), sh[(deg+1)^2 * 3][n] with plane index
  coef * 3 + channel and coefficients ordered l = 0..deg, m = -l..l.
"""
from __future__ import annotations

import dataclasses
import math

import numpy as np

# Real spherical harmonic Y_0^0 = 1 / (2 sqrt(pi)); only used to turn a
# requested base colour into the degree-0 coefficient of a scene.
_Y00 = 0.5 / math.sqrt(math.pi)


@dataclasses.dataclass
class Camera:
    width: int
    height: int
    fx: float
    fy: float
    cx: float
    cy: float
    R: np.ndarray  # (3, 3) float64, camera-to-world rotation, columns = camera axes in world
    t: np.ndarray  # (3,) float64, camera centre in world
    z_near: float = 0.2
    z_far: float = 100.0

    def copy(self) -> "Camera":
        return dataclasses.replace(self, R=self.R.copy(), t=self.t.copy())


@dataclasses.dataclass
class Scene:
    n: int
    sh_degree: int
    pos: np.ndarray      # (3, n) float32
    quat: np.ndarray     # (4, n) float32
    scale: np.ndarray    # (2, n) float32
    opacity: np.ndarray  # (n,) float32
    sh: np.ndarray       # ((deg+1)^2 * 3, n) float32

    def arrays(self):
        return dict(pos=self.pos, quat=self.quat, scale=self.scale,
                    opacity=self.opacity, sh=self.sh)

    def subset(self, idx) -> "Scene":
        idx = np.asarray(idx)
        return Scene(len(idx), self.sh_degree,
                     np.ascontiguousarray(self.pos[:, idx]),
                     np.ascontiguousarray(self.quat[:, idx]),
                     np.ascontiguousarray(self.scale[:, idx]),
                     np.ascontiguousarray(self.opacity[idx]),
                     np.ascontiguousarray(self.sh[:, idx]))


def look_at(eye, target, up, width, height, fx, fy=None, cx=None, cy=None,
            z_near=0.2, z_far=100.0) -> Camera:
    """Pinhole camera at `eye` looking at `target`; `up` is a world vector
    that ends up pointing towards -y (image up)."""
    eye = np.asarray(eye, np.float64)
    z = np.asarray(target, np.float64) - eye
    z /= np.linalg.norm(z)
    x = np.cross(z, np.asarray(up, np.float64))
    x /= np.linalg.norm(x)
    y = np.cross(z, x)
    R = np.stack([x, y, z], axis=1)
    fy = fx if fy is None else fy
    cx = (width - 1) / 2.0 if cx is None else cx
    cy = (height - 1) / 2.0 if cy is None else cy
    return Camera(int(width), int(height), float(fx), float(fy), float(cx),
                  float(cy), R, eye.copy(), z_near, z_far)


def affiliated(cam: Camera, baseline: float) -> Camera:
    """Affiliated eye of a stereo rig: same orientation, centre moved by
    `baseline` along the dominant camera's x axis."""
    c = cam.copy()
    c.t = cam.t + baseline * cam.R[:, 0]
    return c


def _sigmoid(x):
    return 1.0 / (1.0 + np.exp(-x))


def _unit_quats(rng, n):
    q = rng.normal(size=(n, 4))
    q /= np.linalg.norm(q, axis=1, keepdims=True)
    return q


def _quat_from_frames(tu, tv, tw):
    """Unit quaternions (w, x, y, z) of rotations whose columns are tu, tv, tw."""
    m = np.stack([tu, tv, tw], axis=2)  # (n, 3, 3), columns
    n = m.shape[0]
    q = np.empty((n, 4))
    tr = m[:, 0, 0] + m[:, 1, 1] + m[:, 2, 2]
    # Shepperd's method: pick the largest of the four candidate divisors.
    cand = np.stack([tr, m[:, 0, 0], m[:, 1, 1], m[:, 2, 2]], axis=1)
    which = np.argmax(cand, axis=1)
    for c in range(4):
        s = which == c
        if not np.any(s):
            continue
        a = m[s]
        if c == 0:
            r = np.sqrt(1.0 + tr[s]) * 2.0
            q[s, 0] = 0.25 * r
            q[s, 1] = (a[:, 2, 1] - a[:, 1, 2]) / r
            q[s, 2] = (a[:, 0, 2] - a[:, 2, 0]) / r
            q[s, 3] = (a[:, 1, 0] - a[:, 0, 1]) / r
        elif c == 1:
            r = np.sqrt(1.0 + a[:, 0, 0] - a[:, 1, 1] - a[:, 2, 2]) * 2.0
            q[s, 0] = (a[:, 2, 1] - a[:, 1, 2]) / r
            q[s, 1] = 0.25 * r
            q[s, 2] = (a[:, 0, 1] + a[:, 1, 0]) / r
            q[s, 3] = (a[:, 0, 2] + a[:, 2, 0]) / r
        elif c == 2:
            r = np.sqrt(1.0 + a[:, 1, 1] - a[:, 0, 0] - a[:, 2, 2]) * 2.0
            q[s, 0] = (a[:, 0, 2] - a[:, 2, 0]) / r
            q[s, 1] = (a[:, 0, 1] + a[:, 1, 0]) / r
            q[s, 2] = 0.25 * r
            q[s, 3] = (a[:, 1, 2] + a[:, 2, 1]) / r
        else:
            r = np.sqrt(1.0 + a[:, 2, 2] - a[:, 0, 0] - a[:, 1, 1]) * 2.0
            q[s, 0] = (a[:, 1, 0] - a[:, 0, 1]) / r
            q[s, 1] = (a[:, 0, 2] + a[:, 2, 0]) / r
            q[s, 2] = (a[:, 1, 2] + a[:, 2, 1]) / r
            q[s, 3] = 0.25 * r
    q /= np.linalg.norm(q, axis=1, keepdims=True)
    return q


def _uniform_dirs(rng, n):
    d = rng.normal(size=(n, 3))
    d /= np.linalg.norm(d, axis=1, keepdims=True)
    return d


def _pack(pos, quat, scale, opacity, sh, deg) -> Scene:
    n = pos.shape[0]
    nc = (deg + 1) ** 2
    sh = np.asarray(sh, np.float64).reshape(n, nc * 3)
    return Scene(
        n, deg,
        np.ascontiguousarray(pos.T, dtype=np.float32),
        np.ascontiguousarray(quat.T, dtype=np.float32),
        np.ascontiguousarray(scale.T, dtype=np.float32),
        np.ascontiguousarray(opacity, dtype=np.float32),
        np.ascontiguousarray(sh.T, dtype=np.float32))


def scene_uniform_cube(seed: int, n: int = 10_000, half: float = 1.0,
                       log_scale=(-3.5, 0.5), opacity_logit=(0.0, 1.5)) -> Scene:
    """Surfels with centres uniform in a cube of side 2*half, uniform random
    rotations (normalised Gaussian quaternions), log-normal scales, opacity
    sigmoid(N(.)) and SH degree 0 colour uniform in [0,1]^3."""
    rng = np.random.default_rng(seed)
    pos = rng.uniform(-half, half, size=(n, 3))
    quat = _unit_quats(rng, n)
    scale = np.exp(rng.normal(log_scale[0], log_scale[1], size=(n, 2)))
    opacity = _sigmoid(rng.normal(opacity_logit[0], opacity_logit[1], size=n))
    rgb = rng.uniform(0.0, 1.0, size=(n, 3))
    sh = (rgb - 0.5) / _Y00
    return _pack(pos, quat, scale, opacity, sh, 0)


def scene_sphere_shell(seed: int, n: int = 300_000, radius: float = 1.0,
                       normal_sigma: float = 0.02, log_scale=(-3.5, 0.5),
                       opacity_logit=(1.0, 1.0), sh_degree: int = 3,
                       sh_sigma: float = 0.2) -> Scene:
    """Object-centric scene: surfels on a noisy sphere shell, tangent to the
    sphere (normal = radial direction) with a uniform in-plane angle."""
    rng = np.random.default_rng(seed)
    d = _uniform_dirs(rng, n)
    r = radius + rng.normal(0.0, normal_sigma, size=n)
    pos = d * r[:, None]
    ang = rng.uniform(0.0, 2.0 * np.pi, size=n)
    ref = np.where(np.abs(d[:, 2:3]) < 0.9, np.array([[0.0, 0.0, 1.0]]),
                   np.array([[1.0, 0.0, 0.0]]))
    u0 = np.cross(ref, d)
    u0 /= np.linalg.norm(u0, axis=1, keepdims=True)
    v0 = np.cross(d, u0)
    tu = np.cos(ang)[:, None] * u0 + np.sin(ang)[:, None] * v0
    tv = np.cross(d, tu)
    quat = _quat_from_frames(tu, tv, d)
    scale = np.exp(rng.normal(log_scale[0], log_scale[1], size=(n, 2)))
    opacity = _sigmoid(rng.normal(opacity_logit[0], opacity_logit[1], size=n))
    nc = (sh_degree + 1) ** 2
    sh = rng.normal(0.0, sh_sigma, size=(n, nc * 3))
    return _pack(pos, quat, scale, opacity, sh, sh_degree)


def scene_unbounded(seed: int, n: int = 1_000_000, inner_frac: float = 0.7,
                    shell=(1.0, 20.0), log_scale=(-3.5, 0.5),
                    opacity_logit=(0.0, 2.0), sh_degree: int = 3,
                    sh_sigma: float = 0.2) -> Scene:
    """Unbounded scene: a fraction of the centres uniform in the unit ball,
    the rest in a shell whose radius is log-uniform; uniform rotations."""
    rng = np.random.default_rng(seed)
    n_in = int(round(n * inner_frac))
    n_out = n - n_in
    d_in = _uniform_dirs(rng, n_in)
    r_in = rng.uniform(0.0, 1.0, size=n_in) ** (1.0 / 3.0)
    d_out = _uniform_dirs(rng, n_out)
    r_out = np.exp(rng.uniform(np.log(shell[0]), np.log(shell[1]), size=n_out))
    pos = np.concatenate([d_in * r_in[:, None], d_out * r_out[:, None]], axis=0)
    quat = _unit_quats(rng, n)
    scale = np.exp(rng.normal(log_scale[0], log_scale[1], size=(n, 2)))
    opacity = _sigmoid(rng.normal(opacity_logit[0], opacity_logit[1], size=n))
    nc = (sh_degree + 1) ** 2
    sh = rng.normal(0.0, sh_sigma, size=(n, nc * 3))
    return _pack(pos, quat, scale, opacity, sh, sh_degree)


# ---------------------------------------------------------------------------
# Workload presets.  Each returns the scene, the list of dominant cameras and
# the stereo baseline; the affiliated eye is `affiliated(cam, baseline)`.
# ---------------------------------------------------------------------------

BASELINE_IPD = 0.064


def workload_cube256(seed: int = 0, n: int = 10_000):
    """10k surfels in the [-1,1]^3 cube, SH0, 256x256 per eye, fx=fy=300,
    dominant eye at distance 4 looking at the origin."""
    scene = scene_uniform_cube(seed, n)
    cam = look_at((0.0, -4.0, 0.0), (0.0, 0.0, 0.0), (0.0, 0.0, 1.0), 256, 256, 300.0)
    return scene, [cam], BASELINE_IPD


def workload_sphere800(seed: int = 0, n: int = 300_000, n_poses: int = 16):
    """300k surfels on a noisy unit sphere shell, SH3, 800x600 per eye,
    fx=fy=1100, dominant poses on an orbit of radius 3."""
    scene = scene_sphere_shell(seed, n)
    cams = []
    for k in range(n_poses):
        th = 2.0 * np.pi * k / n_poses
        eye = (3.0 * np.cos(th), 3.0 * np.sin(th), 0.0)
        cams.append(look_at(eye, (0.0, 0.0, 0.0), (0.0, 0.0, 1.0), 800, 600, 1100.0))
    return scene, cams, BASELINE_IPD


def workload_unbounded1600(seed: int = 0, n: int = 1_000_000, n_poses: int = 32):
    """1M surfels (70% unit ball, 30% log-uniform shell of radius 1-20), SH3,
    1600x1064 per eye, fx=fy=1300, poses along a forward trajectory."""
    scene = scene_unbounded(seed, n)
    cams = []
    for k in range(n_poses):
        y = -6.0 + 4.5 * k / max(n_poses - 1, 1)
        eye = (0.0, y, 0.0)
        cams.append(look_at(eye, (0.0, y + 1.0, 0.0), (0.0, 0.0, 1.0), 1600, 1064, 1300.0))
    return scene, cams, BASELINE_IPD


def workload_serve2064(seed: int = 0, n: int = 1_000_000, n_poses: int = 32):
    """The serving workload: the unbounded 1M-surfel SH3 scene seen at
    2064x2208 per eye (fx=fy=1700), poses along the forward trajectory."""
    scene = scene_unbounded(seed, n)
    cams = []
    for k in range(n_poses):
        y = -6.0 + 4.5 * k / max(n_poses - 1, 1)
        eye = (0.0, y, 0.0)
        cams.append(look_at(eye, (0.0, y + 1.0, 0.0), (0.0, 0.0, 1.0), 2064, 2208, 1700.0))
    return scene, cams, BASELINE_IPD


BATCH_RESOLUTIONS = ((640, 480), (1024, 768), (1440, 1600), (1920, 1080))


def workload_batch(seed: int = 0, n_pairs: int = 64, sizes=(50_000, 200_000, 600_000, 1_200_000)):
    """The batched configuration: four resident scenes, cube type (uniform
    in [-1,1]^3, SH0, as the 10k cube scene) for the 1st and 3rd size and
    shell type (noisy unit sphere shell, SH3, as the 300k scene) for the
    2nd and 4th, and n_pairs stereo pairs, pair i on scene i mod 4, each
    with a resolution drawn from BATCH_RESOLUTIONS and fx = fy = 1.17 W
    (cube type: 300 / 256) or 1.375 W (shell type: 1100 / 800).  Cube-type
    eyes sit at distance 4 from the origin and shell-type eyes on an orbit
    of radius 3, at seeded azimuths, all looking at the origin.  Returns
    (scenes, [(scene index, dominant camera)], baseline)."""
    scenes = [scene_uniform_cube(seed, sizes[0]), scene_sphere_shell(seed + 1, sizes[1]),
              scene_uniform_cube(seed + 2, sizes[2]), scene_sphere_shell(seed + 3, sizes[3])]
    rng = np.random.default_rng(seed + 100)
    pairs = []
    for i in range(n_pairs):
        si = i % 4
        W, H = BATCH_RESOLUTIONS[int(rng.integers(0, len(BATCH_RESOLUTIONS)))]
        th = float(rng.uniform(0.0, 2.0 * np.pi))
        if si % 2 == 0:
            eye = (4.0 * np.sin(th), -4.0 * np.cos(th), float(rng.uniform(-0.5, 0.5)))
            fx = 1.17 * W
        else:
            eye = (3.0 * np.cos(th), 3.0 * np.sin(th), float(rng.uniform(-0.3, 0.3)))
            fx = 1.375 * W
        pairs.append((si, look_at(eye, (0.0, 0.0, 0.0), (0.0, 0.0, 1.0), W, H, fx)))
    return scenes, pairs, BASELINE_IPD


WORKLOADS = {
    "cube256": workload_cube256,
    "sphere800": workload_sphere800,
    "unbounded1600": workload_unbounded1600,
    "serve2064": workload_serve2064,
}


# ---------------------------------------------------------------------------
# Hand-built scenes for closed-form checks.
# ---------------------------------------------------------------------------

def explicit_scene(pos, tu, tv, su, sv, opacity, rgb) -> Scene:
    """Scene from explicit centres, tangent frames, scales, opacities and
    base colours (degree-0 SH)."""
    pos = np.atleast_2d(np.asarray(pos, np.float64))
    tu = np.atleast_2d(np.asarray(tu, np.float64))
    tv = np.atleast_2d(np.asarray(tv, np.float64))
    tu = tu / np.linalg.norm(tu, axis=1, keepdims=True)
    tv = tv / np.linalg.norm(tv, axis=1, keepdims=True)
    tw = np.cross(tu, tv)
    quat = _quat_from_frames(tu, tv, tw)
    scale = np.stack([np.atleast_1d(su), np.atleast_1d(sv)], axis=1).astype(np.float64)
    opacity = np.atleast_1d(np.asarray(opacity, np.float64))
    rgb = np.atleast_2d(np.asarray(rgb, np.float64))
    sh = (rgb - 0.5) / _Y00
    return _pack(pos, quat, scale, opacity, sh, 0)


def empty_scene(sh_degree: int = 0) -> Scene:
    nc = (sh_degree + 1) ** 2
    return Scene(0, sh_degree, np.zeros((3, 0), np.float32), np.zeros((4, 0), np.float32),
                 np.zeros((2, 0), np.float32), np.zeros((0,), np.float32),
                 np.zeros((nc * 3, 0), np.float32))


# ---------------------------------------------------------------------------
# Stage-level inputs: a dominant-eye image triple (RGB, unnormalised depth
# D = sum d_i w_i, accumulated weight A = sum w_i) with piecewise-planar
# depth, foreground occluders and empty background, so that reprojection,
# hole classification and patching can be fed identical inputs on both
# sides without either side rendering them.
# ---------------------------------------------------------------------------

def stage_images(width: int, height: int, seed: int, n_occluders: int = 6,
                 z_back=(3.0, 6.0), z_front=(0.6, 2.0), bg_frac: float = 0.1):
    rng = np.random.default_rng(seed)
    H, W = height, width
    jj, ii = np.mgrid[0:H, 0:W].astype(np.float64)
    # Background plane with a gentle slope.
    z0 = rng.uniform(*z_back)
    gx, gy = rng.uniform(-0.3, 0.3, size=2)
    z = z0 * (1.0 + gx * (ii / W - 0.5) + gy * (jj / H - 0.5))
    rgb = np.empty((3, H, W))
    base = rng.uniform(0.2, 0.8, size=3)
    for c in range(3):
        rgb[c] = base[c] + 0.15 * np.sin(ii * rng.uniform(0.02, 0.2) + c) * np.cos(jj * rng.uniform(0.02, 0.2))
    alpha = np.ones((H, W))
    # Occluders: axis-aligned rectangles and discs at nearer depth.
    for _ in range(n_occluders):
        zf = rng.uniform(*z_front)
        col = rng.uniform(0.0, 1.0, size=3)
        if rng.uniform() < 0.5:
            x0, x1 = sorted(rng.integers(0, W, size=2))
            y0, y1 = sorted(rng.integers(0, H, size=2))
            m = (ii >= x0) & (ii <= x1) & (jj >= y0) & (jj <= y1)
        else:
            cx0, cy0 = rng.uniform(0, W), rng.uniform(0, H)
            rr = rng.uniform(0.03, 0.2) * min(W, H)
            m = (ii - cx0) ** 2 + (jj - cy0) ** 2 <= rr * rr
        z = np.where(m, zf, z)
        for c in range(3):
            rgb[c] = np.where(m, col[c], rgb[c])
    # Empty background: a blob with alpha 0 and partially covered fringe.
    if bg_frac > 0:
        cx0, cy0 = rng.uniform(0, W), rng.uniform(0, H)
        rr = np.sqrt(bg_frac * W * H / np.pi)
        d2 = ((ii - cx0) ** 2 + (jj - cy0) ** 2) / (rr * rr)
        alpha = np.clip(1.5 * (d2 - 0.5), 0.0, 1.0) * alpha
    # Light multiplicative noise on the weight, never above 1.
    alpha = np.where(alpha > 0, np.clip(alpha * rng.uniform(0.97, 1.0, size=alpha.shape), 0, 1), 0.0)
    rgb = np.clip(rgb * alpha + (1 - alpha) * 0.0, 0.0, 1.0)
    depth_raw = z * alpha
    return (np.ascontiguousarray(rgb, np.float32),
            np.ascontiguousarray(depth_raw, np.float32),
            np.ascontiguousarray(alpha, np.float32))


def random_mask(width: int, height: int, seed: int, density: float) -> np.ndarray:
    rng = np.random.default_rng(seed)
    return (rng.uniform(size=(height, width)) < density).astype(np.uint8)


def serpentine_mask(width: int, height: int) -> np.ndarray:
    """One long one-pixel-wide serpentine: even rows are full, odd rows hold
    a single connector pixel alternating between the right and left ends.
    It is a single component whose label must travel the whole image."""
    m = np.zeros((height, width), np.uint8)
    m[0::2, :] = 1
    for k, j in enumerate(range(1, height, 2)):
        m[j, width - 1 if k % 2 == 0 else 0] = 1
    return m


def checkerboard_mask(width: int, height: int) -> np.ndarray:
    jj, ii = np.mgrid[0:height, 0:width]
    return ((ii + jj) % 2 == 0).astype(np.uint8)


def random_sort_keys(n: int, seed: int, key_bits: int, dup_frac: float = 0.5):
    """Keys with heavy duplication plus values equal to the input position."""
    rng = np.random.default_rng(seed)
    hi = (1 << key_bits) - 1 if key_bits < 32 else 0xFFFFFFFF
    pool = rng.integers(0, hi + 1, size=max(1, int(n * (1 - dup_frac)) + 1), dtype=np.uint64)
    keys = pool[rng.integers(0, len(pool), size=n)].astype(np.uint32)
    vals = np.arange(n, dtype=np.uint32)
    return keys, vals
