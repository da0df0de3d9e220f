"""Seeded synthetic scene generator.

Holds none of the rasterizer's arithmetic: it only draws inputs.  Both the
HIP path and the CPU oracle are fed from here (the oracle through the tests),
so the two sides always see bit-identical FP32 values.

Distributions follow the workloads the paper's method is run on (indoor
RGB-D scenes seen by a pinhole camera, Sec. 4 "Datasets"); the datasets are
absent, so Gaussians are spread uniformly through the camera frustum volume:

* means     : z = cbrt(1 + 124 U) (uniform in volume between 1 m and 5 m),
              pixel (u, v) ~ U(0, W) x U(0, H), back-projected through the
              intrinsics: x = (u - cx) z / fx, y = (v - cy) z / fy
* log-scale : N(-3, 0.5) per axis
* quaternion: normalize(N(0, I4)), stored (w, x, y, z)
* opacity   : logit ~ N(0, 1)  (the kernel applies the sigmoid)
* rgb       : U(0, 1)
* features  : N(0, 1)

Draw order is fixed: means, log-scales, quaternions, opacity logits, rgb,
features, targets, pose noise.  Arrays come back in the layout of the C ABI:
per-Gaussian vectors planar ``[k, P]`` and features row-major ``[P, C]``.
"""
from __future__ import annotations

import dataclasses
import math

import numpy as np


@dataclasses.dataclass
class Camera:
    width: int
    height: int
    fx: float
    fy: float
    cx: float
    cy: float
    viewmat: np.ndarray  # [3, 4] float32, world -> camera, row-major

    def intrinsics(self):
        return (self.width, self.height, self.fx, self.fy, self.cx, self.cy)


@dataclasses.dataclass
class Scene:
    means: np.ndarray          # [3, P] float32
    log_scales: np.ndarray     # [3, P] float32
    quats: np.ndarray          # [4, P] float32 (w, x, y, z)
    logit_opacity: np.ndarray  # [P] float32
    rgb: np.ndarray            # [3, P] float32
    feat: np.ndarray           # [P, C] float32
    camera: Camera

    @property
    def P(self) -> int:
        return int(self.means.shape[1])

    @property
    def C(self) -> int:
        return int(self.feat.shape[1])


# --------------------------------------------------------------------------
# small helpers that only build inputs
# --------------------------------------------------------------------------

def identity_viewmat() -> np.ndarray:
    v = np.zeros((3, 4), dtype=np.float32)
    v[0, 0] = v[1, 1] = v[2, 2] = 1.0
    return v


def _skew(w):
    return np.array([[0.0, -w[2], w[1]], [w[2], 0.0, -w[0]], [-w[1], w[0], 0.0]])


def se3_exp(delta) -> np.ndarray:
    """4x4 homogeneous transform Exp(delta), delta = (rho, theta), FP64.

    Rodrigues' formula for the rotation and the left Jacobian V for the
    translation (standard closed form of the SE(3) exponential)."""
    rho = np.asarray(delta[:3], dtype=np.float64)
    th = np.asarray(delta[3:], dtype=np.float64)
    a = float(np.linalg.norm(th))
    K = _skew(th)
    if a < 1e-12:
        R = np.eye(3) + K
        V = np.eye(3) + 0.5 * K
    else:
        R = np.eye(3) + math.sin(a) / a * K + (1 - math.cos(a)) / a**2 * (K @ K)
        V = (np.eye(3) + (1 - math.cos(a)) / a**2 * K
             + (a - math.sin(a)) / a**3 * (K @ K))
    T = np.eye(4)
    T[:3, :3] = R
    T[:3, 3] = V @ rho
    return T


def perturbed_viewmat(rng, base: np.ndarray, trans_m: float, rot_deg: float):
    """Left-perturb ``base`` (3x4) by Exp(delta0) with |rho| = trans_m and
    |theta| = rot_deg degrees along seeded uniformly random axes."""
    a = rng.normal(size=3)
    a /= np.linalg.norm(a)
    b = rng.normal(size=3)
    b /= np.linalg.norm(b)
    delta = np.concatenate([a * trans_m, b * math.radians(rot_deg)])
    B = np.eye(4)
    B[:3, :] = base.astype(np.float64)
    T = se3_exp(delta) @ B
    return T[:3, :].astype(np.float32), delta


def round_bf16(x: np.ndarray) -> np.ndarray:
    """FP32 -> BF16 bit patterns (uint16), round to nearest even."""
    u = np.ascontiguousarray(x, dtype=np.float32).view(np.uint32).astype(np.uint64)
    lsb = (u >> 16) & 1
    r = ((u + 0x7FFF + lsb) >> 16).astype(np.uint16)
    nan = np.isnan(x)
    if np.any(nan):
        r = r.copy()
        r[nan] = 0x7FC0
    return r


def bf16_to_f32(b: np.ndarray) -> np.ndarray:
    return (np.asarray(b, dtype=np.uint16).astype(np.uint32) << 16).view(np.float32)


def round_f16(x: np.ndarray) -> np.ndarray:
    return np.asarray(x, dtype=np.float32).astype(np.float16)


# --------------------------------------------------------------------------
# scenes
# --------------------------------------------------------------------------

def make_scene(P: int, width: int, height: int, fx: float, fy: float,
               cx: float, cy: float, C: int, seed: int,
               viewmat: np.ndarray | None = None,
               rng: np.random.Generator | None = None) -> Scene:
    rng = np.random.default_rng(seed) if rng is None else rng
    # means: uniform in the frustum volume at 1-5 m
    z = np.cbrt(1.0 + 124.0 * rng.random(P))
    u = rng.random(P) * width
    v = rng.random(P) * height
    x = (u - cx) * z / fx
    y = (v - cy) * z / fy
    means = np.stack([x, y, z]).astype(np.float32)
    log_scales = rng.normal(-3.0, 0.5, size=(3, P)).astype(np.float32)
    q = rng.normal(size=(4, P))
    q /= np.linalg.norm(q, axis=0, keepdims=True)
    quats = q.astype(np.float32)
    logit = rng.normal(size=P).astype(np.float32)
    rgb = rng.random((3, P)).astype(np.float32)
    feat = rng.normal(size=(P, C)).astype(np.float32)
    cam = Camera(width, height, float(fx), float(fy), float(cx), float(cy),
                 identity_viewmat() if viewmat is None else viewmat)
    return Scene(np.ascontiguousarray(means), np.ascontiguousarray(log_scales),
                 np.ascontiguousarray(quats), logit, np.ascontiguousarray(rgb),
                 np.ascontiguousarray(feat), cam)


def make_targets(rng: np.random.Generator, width: int, height: int, C: int):
    """Seeded L1 targets: RGB ~ U(0,1), depth ~ U(1,5), features ~ N(0,1),
    planar image layout ([3,H,W], [H,W], [C,H,W])."""
    t_rgb = rng.random((3, height, width)).astype(np.float32)
    t_depth = rng.uniform(1.0, 5.0, size=(height, width)).astype(np.float32)
    t_feat = rng.normal(size=(C, height, width)).astype(np.float32)
    return t_rgb, t_depth, t_feat


def upstream_signs(rng: np.random.Generator, width: int, height: int, C: int,
                   with_feat: bool = True):
    """A seeded upstream gradient shaped like the L1 gradient sign(.)/numel of
    each output group (RGB, depth, alpha, features).  Parity tests feed the
    same tensor to both sides so no sign can differ between them."""
    HW = width * height

    def s(shape, n):
        return (rng.integers(0, 2, size=shape) * 2 - 1).astype(np.float32) / n

    g_rgb = s((3, height, width), 3 * HW)
    g_depth = s((height, width), HW)
    g_alpha = s((height, width), HW)
    g_feat = s((C, height, width), max(1, C) * HW) if with_feat else None
    return g_rgb, g_depth, g_alpha, g_feat


# The five workloads the rasterizer is measured on.  ``tiny`` is small enough
# for the FP64 oracle in seconds; ``frame`` is the 640x480 / 200k-Gaussian
# tracking-and-mapping frame the headline throughput is quoted on.
WORKLOADS = {
    "tiny": dict(P=2_000, width=64, height=48, fx=50.0, fy=50.0, cx=32.0, cy=24.0,
                 C=16, seed=1),
    "frame": dict(P=200_000, width=640, height=480, fx=525.0, fy=525.0, cx=320.0,
                  cy=240.0, C=16, seed=2),
    "mixed": dict(P=1_000_000, width=1200, height=680, fx=600.0, fy=600.0,
                  cx=600.0, cy=340.0, C=64, seed=3),
    "decoder": dict(P=500_000, width=640, height=480, fx=525.0, fy=525.0,
                    cx=320.0, cy=240.0, C=16, seed=4),
}


def workload_scene(name: str, perturb_pose: bool | None = None,
                   P: int | None = None):
    """Scene for a named workload.  For ``frame`` the camera is the identity
    pose left-perturbed by 1 cm / 1 degree on seeded random axes (the
    tracking situation); ``P`` overrides the Gaussian count (for scaled-down
    cases with the same distributions)."""
    cfg = dict(WORKLOADS[name])
    seed = cfg.pop("seed")
    if P is not None:
        cfg["P"] = P
    rng = np.random.default_rng(seed)
    scene = make_scene(rng=rng, seed=seed, **cfg)
    if perturb_pose is None:
        perturb_pose = name == "frame"
    if perturb_pose:
        # pose noise is drawn after the scene (and after targets, which the
        # caller draws from the returned generator if it needs them)
        prng = np.random.default_rng(seed + 1000)
        vm, _ = perturbed_viewmat(prng, identity_viewmat(), 0.01, 1.0)
        scene.camera.viewmat = vm
    return scene, rng


# --------------------------------------------------------------------------
# multi-view and semantic inputs
# --------------------------------------------------------------------------

def look_at_viewmat(cam_pos, target) -> np.ndarray:
    """3x4 world->camera matrix of a camera at cam_pos looking at target, with
    camera y pointing down along world +y (OpenCV axes)."""
    c = np.asarray(cam_pos, np.float64)
    z = np.asarray(target, np.float64) - c
    z /= np.linalg.norm(z)
    y0 = np.array([0.0, 1.0, 0.0])
    x = np.cross(y0, z)
    x /= np.linalg.norm(x)
    y = np.cross(z, x)
    R = np.stack([x, y, z])
    V = np.zeros((3, 4))
    V[:, :3] = R
    V[:, 3] = -R @ c
    return V


def arc_viewmats(rng, n_views: int, radius: float = 3.0, arc: float = 2.0,
                 center=(0.0, 0.0, 3.0), jitter_deg: float = 2.0):
    """Cameras on a horizontal circular arc of the given length around
    `center`, centred on the reference camera at the origin, each looking at
    the centre, then left-perturbed by a seeded rotation of up to jitter_deg."""
    half = 0.5 * arc / radius
    angles = np.linspace(-half, half, n_views) if n_views > 1 else np.zeros(1)
    c = np.asarray(center, np.float64)
    out = []
    for phi in angles:
        pos = c + radius * np.array([np.sin(phi), 0.0, -np.cos(phi)])
        V = look_at_viewmat(pos, c)
        if jitter_deg > 0:
            V, _ = perturbed_viewmat(rng, V.astype(np.float32), 0.0, jitter_deg)
        out.append(np.asarray(V, np.float32))
    return out


def semantic_features(rng, means: np.ndarray, n_classes: int = 32, dim: int = 512,
                      noise: float = 0.05):
    """Class-structured high-dimensional features standing in for text
    embeddings of labelled regions: n_classes seeded unit query vectors q_k,
    class centres at n_classes seeded Gaussian means, every Gaussian takes the
    class of its nearest centre and the feature normalize(q_k + noise xi).
    Returns (feat [P, dim] float32, labels [P] int32, queries [n_classes, dim])."""
    P = means.shape[1]
    q = rng.normal(size=(n_classes, dim))
    q /= np.linalg.norm(q, axis=1, keepdims=True)
    centers = means[:, rng.choice(P, n_classes, replace=False)].T.astype(np.float64)
    labels = np.empty(P, dtype=np.int32)
    pts = means.T.astype(np.float64)
    for a in range(0, P, 65536):
        d = ((pts[a:a + 65536, None, :] - centers[None]) ** 2).sum(-1)
        labels[a:a + 65536] = d.argmin(1)
    f = q[labels] + noise * rng.normal(size=(P, dim))
    f /= np.linalg.norm(f, axis=1, keepdims=True)
    return f.astype(np.float32), labels, q.astype(np.float32)
