"""FP64 projection of complex 3D Gaussians and its analytic backward.

Forward (Sec. 3, Eqs. 2-4; Sec. 4.1, Eqs. 8 and 10):
  Sigma   = R S S^T R^T,   R from the normalised quaternion, S = diag(exp(s))
  t       = W x + t0        (W: world-to-camera rotation of the camera)
  J       = d(pixel)/d(t) of the pinhole map  [[fx/tz, 0, -fx tx/tz^2],
                                                [0, fy/tz, -fy ty/tz^2]]
  Sigma'  = J W Sigma W^T J^T     (no low-pass dilation: the paper adds none)
  mu      = (fx tx/tz + cx, fy ty/tz + cy)
  conic   = Sigma'^{-1}
  v_l     = c_l exp(j phi_l)   per wavelength (the field of Eq. 10 without G)

Backward (Supplementary D, backward pass): the chain
  d(mu), d(conic) -> d(Sigma') (matrix-inverse rule) -> d(J), d(Sigma)
  -> d(t) (through mu and J) -> d(x) = W^T d(t);  d(Sigma) -> d(s), d(q).
The supplement's chain for the centre drops the dependence of J on t; it is
kept here (reading listed in the design notes), and finite differences pin it.
"""
from __future__ import annotations

from dataclasses import dataclass

import numpy as np


def quat_to_rotmat(q):
    """Rotation matrices [N,3,3] from quaternions (w, x, y, z) of any norm."""
    q = np.asarray(q, np.float64)
    qn = q / np.linalg.norm(q, axis=1, keepdims=True)
    w, x, y, z = qn.T
    R = np.empty((q.shape[0], 3, 3))
    R[:, 0, 0] = 1 - 2 * (y * y + z * z)
    R[:, 0, 1] = 2 * (x * y - w * z)
    R[:, 0, 2] = 2 * (x * z + w * y)
    R[:, 1, 0] = 2 * (x * y + w * z)
    R[:, 1, 1] = 1 - 2 * (x * x + z * z)
    R[:, 1, 2] = 2 * (y * z - w * x)
    R[:, 2, 0] = 2 * (x * z - w * y)
    R[:, 2, 1] = 2 * (y * z + w * x)
    R[:, 2, 2] = 1 - 2 * (x * x + y * y)
    return R


def _drot_dq(qn):
    """dR/dw, dR/dx, dR/dy, dR/dz at unit quaternions: array [N,4,3,3]."""
    w, x, y, z = qn.T
    o = np.zeros_like(w)
    d = np.empty((qn.shape[0], 4, 3, 3))
    d[:, 0] = 2 * np.stack([np.stack([o, -z, y], -1), np.stack([z, o, -x], -1), np.stack([-y, x, o], -1)], 1)
    d[:, 1] = 2 * np.stack([np.stack([o, y, z], -1), np.stack([y, -2 * x, -w], -1), np.stack([z, w, -2 * x], -1)], 1)
    d[:, 2] = 2 * np.stack([np.stack([-2 * y, x, w], -1), np.stack([x, o, z], -1), np.stack([-w, z, -2 * y], -1)], 1)
    d[:, 3] = 2 * np.stack([np.stack([-2 * z, -w, x], -1), np.stack([w, -2 * z, y], -1), np.stack([x, y, o], -1)], 1)
    return d


@dataclass
class ProjectedGaussians:
    t: np.ndarray        # [N,3] camera-space centres
    J: np.ndarray        # [N,2,3]
    M: np.ndarray        # [N,3,3] camera-space 3D covariance W Sigma W^T
    cov2d: np.ndarray    # [N,2,2] Sigma'
    mu: np.ndarray       # [N,2] pixel coordinates of the centre
    conic: np.ndarray    # [N,3] (A, B, C) of Sigma'^{-1} = [[A, B], [B, C]]
    v: np.ndarray        # [N,L] complex128 amplitude * exp(j phase)
    Rq: np.ndarray       # [N,3,3]
    scale2: np.ndarray   # [N,3] exp(2 s)


def project(means, log_scales, quats, amp, phase, cam) -> ProjectedGaussians:
    m = np.asarray(means, np.float64)
    s = np.asarray(log_scales, np.float64)
    W = np.asarray(cam.R, np.float64).reshape(3, 3)
    t0 = np.asarray(cam.t, np.float64)
    fx, fy, cx, cy = (float(np.float32(v)) for v in (cam.fx, cam.fy, cam.cx, cam.cy))
    Rq = quat_to_rotmat(quats)
    s2 = np.exp(2.0 * s)
    Sigma = np.einsum("nij,nj,nkj->nik", Rq, s2, Rq)
    t = m @ W.T + t0
    tx, ty, tz = t.T
    with np.errstate(all="ignore"):
        J = np.zeros((m.shape[0], 2, 3))
        J[:, 0, 0] = fx / tz
        J[:, 0, 2] = -fx * tx / tz ** 2
        J[:, 1, 1] = fy / tz
        J[:, 1, 2] = -fy * ty / tz ** 2
        M = np.einsum("ij,njk,lk->nil", W, Sigma, W)
        cov2d = np.einsum("nij,njk,nlk->nil", J, M, J)
        mu = np.stack([fx * tx / tz + cx, fy * ty / tz + cy], axis=1)
        det = cov2d[:, 0, 0] * cov2d[:, 1, 1] - cov2d[:, 0, 1] ** 2
        conic = np.stack([cov2d[:, 1, 1] / det, -cov2d[:, 0, 1] / det, cov2d[:, 0, 0] / det], axis=1)
    v = np.asarray(amp, np.float64) * np.exp(1j * np.asarray(phase, np.float64))
    return ProjectedGaussians(t, J, M, cov2d, mu, conic, v, Rq, s2)


def project_backward(p: ProjectedGaussians, quats, amp, phase, cam, d_mu, d_conic, d_opacity, d_v):
    """Chain per-view 2D gradients to the 3D parameters of every Gaussian.

    d_mu [N,2], d_conic [N,3] (w.r.t. the scalars A, B, C of the conic, where B
    appears in both off-diagonal slots), d_opacity [N], d_v [N,L] complex with
    the convention dL/dRe + j dL/dIm.  Returns a dict of FP64 arrays shaped
    like the parameters.
    """
    W = np.asarray(cam.R, np.float64).reshape(3, 3)
    fx, fy = float(np.float32(cam.fx)), float(np.float32(cam.fy))
    q = np.asarray(quats, np.float64)
    qnorm = np.linalg.norm(q, axis=1, keepdims=True)
    qn = q / qnorm
    A, B, C = p.conic.T
    Q = np.stack([np.stack([A, B], -1), np.stack([B, C], -1)], 1)
    dA, dB, dC = np.asarray(d_conic, np.float64).T
    GQ = np.stack([np.stack([dA, 0.5 * dB], -1), np.stack([0.5 * dB, dC], -1)], 1)
    Gcov = -np.einsum("nij,njk,nkl->nil", Q, GQ, Q)
    GM = np.einsum("nji,njk,nkl->nil", p.J, Gcov, p.J)             # J^T G J
    GJ = 2.0 * np.einsum("nij,njk,nkl->nil", Gcov, p.J, p.M)        # 2 G J M
    GSigma = np.einsum("ji,njk,kl->nil", W, GM, W)                  # W^T GM W
    # scales: Sigma = Rq diag(s2) Rq^T
    RtGR = np.einsum("nji,njk,nkl->nil", p.Rq, GSigma, p.Rq)
    d_logs = 2.0 * p.scale2 * np.einsum("nii->ni", RtGR)
    GRq = 2.0 * np.einsum("nij,njk,nk->nik", GSigma, p.Rq, p.scale2)
    dqn = np.einsum("nij,nkij->nk", GRq, _drot_dq(qn))
    d_q = (dqn - qn * np.sum(qn * dqn, axis=1, keepdims=True)) / qnorm
    # centre: through mu and through J
    tx, ty, tz = p.t.T
    dmx, dmy = np.asarray(d_mu, np.float64).T
    dt = np.zeros_like(p.t)
    dt[:, 0] = dmx * fx / tz + GJ[:, 0, 2] * (-fx / tz ** 2)
    dt[:, 1] = dmy * fy / tz + GJ[:, 1, 2] * (-fy / tz ** 2)
    dt[:, 2] = (-dmx * fx * tx / tz ** 2 - dmy * fy * ty / tz ** 2
                + GJ[:, 0, 0] * (-fx / tz ** 2) + GJ[:, 0, 2] * (2 * fx * tx / tz ** 3)
                + GJ[:, 1, 1] * (-fy / tz ** 2) + GJ[:, 1, 2] * (2 * fy * ty / tz ** 3))
    d_means = dt @ W
    ph = np.asarray(phase, np.float64)
    am = np.asarray(amp, np.float64)
    d_amp = d_v.real * np.cos(ph) + d_v.imag * np.sin(ph)
    d_phase = am * (-d_v.real * np.sin(ph) + d_v.imag * np.cos(ph))
    return {"means": d_means, "log_scales": d_logs, "quats": d_q,
            "opacity": np.asarray(d_opacity, np.float64), "amp": d_amp, "phase": d_phase}
