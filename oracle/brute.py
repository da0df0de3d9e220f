"""Pure-numpy FP64 brute force of the rasterizer's forward (test
infrastructure only).

Written independently of ``gsff_oracle.cpp`` to validate it on tiny scenes:
rotations come from the quaternion sandwich product q v q* instead of the
closed-form matrix, the covariance is assembled as a sum of scaled outer
products of the rotated axes, the conic comes from a general matrix inverse,
and every Gaussian is evaluated at every pixel with no bounding box at all.
Blending follows Eqs. 2-3 of the paper with the readings stated in the oracle.
"""
from __future__ import annotations

import numpy as np


def _qmul(a, b):
    aw, ax, ay, az = a
    bw, bx, by, bz = b
    return np.array([aw * bw - ax * bx - ay * by - az * bz,
                     aw * bx + ax * bw + ay * bz - az * by,
                     aw * by - ax * bz + ay * bw + az * bx,
                     aw * bz + ax * by - ay * bx + az * bw])


def _rotate(q, v):
    qc = np.array([q[0], -q[1], -q[2], -q[3]])
    return _qmul(_qmul(q, np.concatenate([[0.0], v])), qc)[1:]


def splats(params, camera, near=0.2, guard=1.3, dilation=0.3, alpha_min=1 / 255,
           alpha_max=0.99):
    """Every Gaussian the culling rules keep, in blending order ((depth key,
    index) ascending), evaluated at every pixel centre with no bounding box:
    dict ids [n], alpha [n, H*W] (clamped at alpha_max, not yet thresholded),
    depth [n], rx / ry [n] (half-widths of the exact box of alpha >= alpha_min,
    from this module's own 2D covariance) and u / v [n]."""
    means = np.asarray(params["means"], np.float64)
    P = means.shape[1]
    logs = np.asarray(params["log_scales"], np.float64)
    quats = np.asarray(params["quats"], np.float64)
    logit = np.asarray(params["logit_opacity"], np.float64)
    W, H = int(camera["width"]), int(camera["height"])
    fx, fy, cx, cy = (float(camera[k]) for k in ("fx", "fy", "cx", "cy"))
    V = np.asarray(camera["viewmat"], np.float64).reshape(3, 4)
    Rv, tv = V[:, :3], V[:, 3]

    ys, xs = np.mgrid[0:H, 0:W]
    pcx = xs.reshape(-1) + 0.5
    pcy = ys.reshape(-1) + 0.5

    keep, alpha_rows, keys, depth, rx, ry, us, vs = [], [], [], [], [], [], [], []
    for i in range(P):
        mw = means[:, i]
        mc = Rv @ mw + tv
        x, y, z = mc
        zk = ((V[2, 0] * mw[0] + V[2, 1] * mw[1]) + V[2, 2] * mw[2]) + V[2, 3]
        if not (z > near):
            continue
        if abs(x / z) > guard * W / (2 * fx) or abs(y / z) > guard * H / (2 * fy):
            continue
        q = quats[:, i]
        n = np.linalg.norm(q)
        if not n > 0:
            continue
        q = q / n
        o = 1.0 / (1.0 + np.exp(-logit[i]))
        s = np.exp(logs[:, i])
        Sig = np.zeros((3, 3))
        for k in range(3):
            e = np.zeros(3)
            e[k] = 1.0
            r = _rotate(q, e)
            Sig += s[k] ** 2 * np.outer(r, r)
        Sc = Rv @ Sig @ Rv.T
        J = np.array([[fx / z, 0.0, -fx * x / z**2], [0.0, fy / z, -fy * y / z**2]])
        S2 = J @ Sc @ J.T + dilation * np.eye(2)
        Kc = np.linalg.inv(S2)
        u = fx * x / z + cx
        v = fy * y / z + cy
        d = np.stack([u - pcx, v - pcy])  # [2, HW]
        power = -0.5 * np.einsum("ip,ij,jp->p", d, Kc, d)
        oG = o * np.exp(power)
        alpha_rows.append(np.minimum(alpha_max, oG))
        keep.append(i)
        keys.append(np.float32(zk))
        depth.append(z)
        k2 = 2.0 * np.log(o / alpha_min) if o > 0 else -1.0
        rx.append(np.sqrt(k2 * S2[0, 0]) if k2 >= 0 else -1.0)
        ry.append(np.sqrt(k2 * S2[1, 1]) if k2 >= 0 else -1.0)
        us.append(u)
        vs.append(v)
    n = len(keep)
    order = np.lexsort((np.array(keep, dtype=np.int64), np.array(keys, dtype=np.float32))) \
        if n else np.zeros(0, dtype=np.int64)
    pick = lambda a, dt=np.float64: np.asarray(a, dt)[order] if n else np.zeros(0, dt)
    return dict(ids=pick(keep, np.int64),
                alpha=np.stack(alpha_rows)[order] if n else np.zeros((0, H * W)),
                depth=pick(depth), rx=pick(rx), ry=pick(ry), u=pick(us), v=pick(vs))


def render(params, camera, near=0.2, guard=1.3, dilation=0.3, alpha_min=1 / 255,
           alpha_max=0.99, t_min=1e-4, render_features=True):
    P = np.asarray(params["means"]).shape[1]
    rgb = np.asarray(params["rgb"], np.float64)
    feat = params.get("feat")
    feat = np.zeros((P, 0)) if feat is None else np.asarray(feat, np.float64)
    C = feat.shape[1]
    W, H = int(camera["width"]), int(camera["height"])
    sp = splats(params, camera, near, guard, dilation, alpha_min, alpha_max)
    HW = H * W
    out_rgb = np.zeros((3, HW))
    out_d = np.zeros(HW)
    out_f = np.zeros((C, HW))
    T = np.ones(HW)
    live = np.ones(HW, dtype=bool)
    for j, i in enumerate(sp["ids"]):
        a = sp["alpha"][j]
        ok = live & (a >= alpha_min)
        Tn = T * (1.0 - a)
        stop = ok & (Tn < t_min)
        live &= ~stop
        ok &= ~stop
        w = np.where(ok, a * T, 0.0)
        out_rgb += rgb[:, i:i + 1] * w
        out_d += sp["depth"][j] * w
        if render_features:
            out_f += feat[i][:, None] * w
        T = np.where(ok, Tn, T)
    return dict(rgb=out_rgb.reshape(3, H, W), depth=out_d.reshape(H, W),
                alpha=(1.0 - T).reshape(H, W), feat=out_f.reshape(C, H, W),
                T=T.reshape(H, W))
