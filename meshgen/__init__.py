"""Seeded synthetic inputs shared by the tests, the oracle checks and bench.py.

This module holds no arithmetic of the integration method: it only draws
element geometry, orders, spaces and arrival times with numpy's PCG64
generator (``numpy.random.default_rng(seed)``).  Both the GPU path and the
oracle receive exactly the arrays produced here.

Layouts (float64, C order):
* trilinear: [E, 8, 3]; vertex v = v1 + 2 v2 + 4 v3 sits at master corner
  (v1, v2, v3).
* affine:    [E, 12]; x0[3] followed by J[3, 3] row-major, J_ij = dx_i/dxi_j.
* extruded:  [E, 10]; x1_0, lambda1, then (x2, x3) of the cross-section corners
  (v2, v3) = (0,0), (1,0), (0,1), (1,1).

The paper measures a single identity-map element and uses no public
dataset; these recipes stand in for the workloads of the benchmark configs.
"""
import numpy as np

SPACE_IDS = {"H1": 0, "HCURL": 1, "HDIV": 2, "L2": 3}
SPACE_NAMES = {v: k for k, v in SPACE_IDS.items()}


def unit_corners():
    """[8, 3] corners of (0,1)^3 in vertex order v = v1 + 2 v2 + 4 v3."""
    v = np.arange(8)
    return np.stack([v & 1, (v >> 1) & 1, (v >> 2) & 1], axis=1).astype(np.float64)


def scaled_cube(scale=2.0):
    """Single cube (0, scale)^3 as a trilinear element, shape [1, 8, 3]."""
    return (scale * unit_corners())[None, :, :].copy()


def perturbed_hexes(n_elem, noise=0.15, seed=1712):
    """Unit-cube vertices plus independent U(-noise, noise) per coordinate."""
    rng = np.random.default_rng(seed)
    base = unit_corners()[None, :, :]
    return base + rng.uniform(-noise, noise, size=(n_elem, 8, 3))


def affine_parallelepipeds(n_elem, shear=0.2, scale_lo=0.5, scale_hi=2.0, seed=1713):
    """J = (I + S) diag(lam): S off-diagonal U(-shear, shear), lam U(lo, hi); x0 = 0."""
    rng = np.random.default_rng(seed)
    S = rng.uniform(-shear, shear, size=(n_elem, 3, 3))
    S[:, np.arange(3), np.arange(3)] = 0.0
    lam = rng.uniform(scale_lo, scale_hi, size=(n_elem, 3))
    J = (np.eye(3)[None] + S) * lam[:, None, :]
    out = np.zeros((n_elem, 12))
    out[:, 3:] = J.reshape(n_elem, 9)
    return out


def affine_as_trilinear(affine):
    """Vertices of the affine maps, for feeding the same elements to the
    trilinear code path: X_v = x0 + J corner_v."""
    affine = np.asarray(affine, dtype=np.float64).reshape(-1, 12)
    x0 = affine[:, :3]
    J = affine[:, 3:].reshape(-1, 3, 3)
    c = unit_corners()
    return x0[:, None, :] + np.einsum("eij,vj->evi", J, c)


def extruded_prisms(n_elem, noise=0.15, lam_lo=0.5, lam_hi=2.0, seed=1716):
    """Quadrilaterals extruded along x1: corners of the unit square plus
    U(-noise, noise) per coordinate, lambda1 ~ U(lo, hi), x1_0 ~ U(-1, 1)."""
    rng = np.random.default_rng(seed)
    out = np.zeros((n_elem, 10))
    out[:, 0] = rng.uniform(-1.0, 1.0, size=n_elem)
    out[:, 1] = rng.uniform(lam_lo, lam_hi, size=n_elem)
    sq = np.array([[0, 0], [1, 0], [0, 1], [1, 1]], dtype=np.float64)
    out[:, 2:] = (sq[None] + rng.uniform(-noise, noise, size=(n_elem, 4, 2))).reshape(n_elem, 8)
    return out


def extruded_as_trilinear(ext):
    """Vertices of the extruded maps, for feeding the same elements to the
    trilinear code path: X_v = (x1_0 + lambda1 v1, q_{v2 v3})."""
    ext = np.asarray(ext, dtype=np.float64).reshape(-1, 10)
    c = unit_corners()
    X = np.zeros((ext.shape[0], 8, 3))
    X[:, :, 0] = ext[:, :1] + ext[:, 1:2] * c[None, :, 0]
    q = ext[:, 2:].reshape(-1, 4, 2)
    corner = (c[:, 1] + 2 * c[:, 2]).astype(int)
    X[:, :, 1:] = q[:, corner, :]
    return X


def mixed_batch(n_elem, p_lo=2, p_hi=9, dp=1, seed=1714, noise=0.15):
    """Uneven batch: space ~ U{H1,HCURL,HDIV,L2}, p ~ U{p_lo..p_hi}, p_r = p + dp."""
    rng = np.random.default_rng(seed)
    space = rng.integers(0, 4, size=n_elem).astype(np.int8)
    p = rng.integers(p_lo, p_hi + 1, size=n_elem)
    pr = (p + dp).astype(np.int8)
    geom = np.random.default_rng(seed + 1000).uniform(-noise, noise, size=(n_elem, 8, 3)) + unit_corners()[None]
    return space, pr, geom


def serving_trace(duration_s=60.0, rate_hz=200.0, n_lo=64, n_hi=2048, p_lo=2, p_hi=10, dp=1, seed=1715):
    """Poisson arrivals: list of dicts(t, space, p, dp, n_elem, seed)."""
    rng = np.random.default_rng(seed)
    t = 0.0
    out = []
    while True:
        t += rng.exponential(1.0 / rate_hz)
        if t >= duration_s:
            break
        out.append(dict(t=t, space=int(rng.integers(0, 4)), p=int(rng.integers(p_lo, p_hi + 1)),
                        dp=dp, n_elem=int(rng.integers(n_lo, n_hi + 1)),
                        seed=int(rng.integers(0, 2**31 - 1))))
    return out
