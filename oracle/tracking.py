"""FP64 numpy oracle of the tracking support (test infrastructure only; only
``tests/`` use it).  Shares no code with the HIP path.

Sec. 3.2 (tracking loss, Eq. 6; camera pose optimisation, Eq. 4):

* ``edge_mask``         -- m_e: Sobel gradient magnitude of the grey target
                           image (mean of r, g, b), scaled by 1/8 so that a ramp
                           of slope a has magnitude a, border replicated; kept
                           where it exceeds the threshold.
* ``visibility_mask``   -- m_v: the render's accumulated opacity above a
                           threshold.
* ``tracking_upstream`` -- the gradient of
                           L = lambda mean(m_v m_e |rgb - t|) + (1 - lambda) mean(m_v |d - t|)
                           with respect to the rendered colour and depth, and L.
* ``se3_exp``           -- the closed-form SE(3) exponential of (rho, theta).
* ``pose_adam_step``    -- one Adam step on the left increment, applied as
                           T <- Exp(delta) T.
* ``relative_motion``   -- rotation angle and translation length of
                           T_now T_then^-1, the net pose change the tracking
                           loop's convergence test measures over a window.

The operator and thresholds of the masks, the means over all elements and
the optimiser (Adam) are readings where the paper gives no detail.
"""
from __future__ import annotations

import numpy as np


def edge_magnitude(t_rgb):
    """|Sobel gradient| / 8 of the grey image of t_rgb [3, H, W]."""
    g = np.asarray(t_rgb, np.float64).mean(axis=0)
    p = np.pad(g, 1, mode="edge")
    # p[1 + y + dy, 1 + x + dx] is the grey value at (x + dx, y + dy)
    def at(dx, dy):
        H, W = g.shape
        return p[1 + dy:1 + dy + H, 1 + dx:1 + dx + W]
    gx = (at(1, -1) + 2 * at(1, 0) + at(1, 1)) - (at(-1, -1) + 2 * at(-1, 0) + at(-1, 1))
    gy = (at(-1, 1) + 2 * at(0, 1) + at(1, 1)) - (at(-1, -1) + 2 * at(0, -1) + at(1, -1))
    return np.hypot(gx, gy) / 8.0


def edge_mask(t_rgb, threshold):
    return edge_magnitude(t_rgb) > threshold


def visibility_mask(alpha, threshold):
    return np.asarray(alpha, np.float64) > threshold


def tracking_upstream(out_rgb, out_depth, t_rgb, t_depth, mask_v, mask_e, lam):
    """(g_rgb [3,H,W], g_depth [H,W], loss) of Eq. 6; None masks keep every
    pixel.  The colour term is weighted by m_v m_e, the depth term by m_v;
    each mean runs over all of its elements (3HW, HW)."""
    o_c = np.asarray(out_rgb, np.float64)
    o_d = np.asarray(out_depth, np.float64)
    H, W = o_d.shape
    mv = np.ones((H, W)) if mask_v is None else (np.asarray(mask_v) != 0).astype(np.float64)
    me = np.ones((H, W)) if mask_e is None else (np.asarray(mask_e) != 0).astype(np.float64)
    r_c = o_c - np.asarray(t_rgb, np.float64)
    r_d = o_d - np.asarray(t_depth, np.float64)
    w_c = lam / (3.0 * H * W) * (mv * me)[None]
    w_d = (1.0 - lam) / (H * W) * mv
    loss = float((w_c * np.abs(r_c)).sum() + (w_d * np.abs(r_d)).sum())
    return w_c * np.sign(r_c), w_d * np.sign(r_d), loss


def hat(v):
    x, y, z = v
    return np.array([[0.0, -z, y], [z, 0.0, -x], [-y, x, 0.0]])


def se3_exp(delta):
    """4x4 matrix Exp(delta), delta = (rho, theta)."""
    rho = np.asarray(delta[:3], np.float64)
    th = np.asarray(delta[3:], np.float64)
    phi = float(np.linalg.norm(th))
    Wm = hat(th)
    W2 = Wm @ Wm
    if phi < 1e-6:
        a, b, c = 1.0 - phi**2 / 6, 0.5 - phi**2 / 24, 1.0 / 6 - phi**2 / 120
    else:
        a = np.sin(phi) / phi
        b = (1.0 - np.cos(phi)) / phi**2
        c = (phi - np.sin(phi)) / phi**3
    T = np.eye(4)
    T[:3, :3] = np.eye(3) + a * Wm + b * W2
    T[:3, 3] = (np.eye(3) + b * Wm + c * W2) @ rho
    return T


def pose_adam_step(viewmat, grad, m, v, step, lr_trans, lr_rot, beta1=0.9, beta2=0.999,
                   eps=1e-8):
    """Returns (viewmat' [3,4], m', v', delta [6])."""
    g = np.asarray(grad, np.float64)
    m = beta1 * np.asarray(m, np.float64) + (1 - beta1) * g
    v = beta2 * np.asarray(v, np.float64) + (1 - beta2) * g * g
    mhat = m / (1 - beta1**step)
    vhat = v / (1 - beta2**step)
    lr = np.array([lr_trans] * 3 + [lr_rot] * 3)
    delta = -lr * mhat / (np.sqrt(vhat) + eps)
    T = np.eye(4)
    T[:3, :] = np.asarray(viewmat, np.float64).reshape(3, 4)
    Tn = se3_exp(delta) @ T
    return Tn[:3, :], m, v, delta


def relative_motion(T_now, T_then):
    """(angle [rad], shift) of the motion T_now T_then^-1 between two 3x4
    world-to-camera poses: the rotation angle of R_now R_then^T (from its
    axis-angle logarithm, ``scipy.spatial.transform``) and the length of its
    translation t_now - R_now R_then^T t_then."""
    from scipy.spatial.transform import Rotation
    A = np.asarray(T_now, np.float64).reshape(3, 4)
    B = np.asarray(T_then, np.float64).reshape(3, 4)
    D = A[:, :3] @ B[:, :3].T
    angle = float(np.linalg.norm(Rotation.from_matrix(D).as_rotvec()))
    shift = float(np.linalg.norm(A[:, 3] - D @ B[:, 3]))
    return angle, shift
