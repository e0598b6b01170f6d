"""The reading behind the FP32 path's vertex-shape routing, checked on the CPU: rounding a
P1 element's edge vectors to FP32 (the FP32 path's only input rounding) moves its stiffness
entries by at most a small multiple of sigma u_32 relative to |T| |grad phi_a| |grad phi_b|,
with sigma = prod_k |e_k| / |det J| the vertex shape seen from the origin node.  So elements
with sigma <= 16 keep that part of the error an order below 1e-5, while on a Delaunay mesh
elements with sigma far above 16 (yet a det-condition far below the default 1e6) exceed 1e-5
from the input rounding alone: the det-condition by itself does not bound the error."""
import numpy as np
import pytest

spatial = pytest.importorskip("scipy.spatial")
U32 = 2.0 ** -24


def _stiffness(e):
    """K_e = |T| G^T G with G the barycentric gradients, from edge rows e (ne, 3, 3) in FP64"""
    J = np.transpose(e, (0, 2, 1))
    Ji = np.linalg.inv(J)  # rows: grad phi_1..3
    g = np.concatenate([-Ji.sum(axis=1, keepdims=True), Ji], axis=1)
    vol = np.abs(np.linalg.det(J)) / 6.0
    K = vol[:, None, None] * np.einsum("eai,ebi->eab", g, g)
    gn = np.linalg.norm(g, axis=2)
    return K, vol[:, None, None] * gn[:, :, None] * gn[:, None, :]


def test_input_rounding_error_scales_with_vertex_shape():
    pts = np.random.default_rng(5).random((20000, 3))
    el = spatial.Delaunay(pts).simplices
    e = pts[el[:, 1:]] - pts[el[:, :1]]
    sigma = np.prod(np.linalg.norm(e, axis=2), axis=1) / np.abs(np.linalg.det(e))
    assert sigma.min() >= 1.0 - 1e-12  # Hadamard's inequality
    K, scale = _stiffness(e)
    K32, _ = _stiffness(e.astype(np.float32).astype(np.float64))
    err = (np.abs(K32 - K) / scale).max(axis=(1, 2))
    assert (err <= 3.0 * sigma * U32).all(), (err / (sigma * U32)).max()
    assert err[sigma <= 16].max() < 2e-6
    bad = err > 1e-5
    assert bad.any() and sigma[bad].min() > 16
    # their det-condition (first-row expansion) is far below the default threshold 1e6
    c1 = np.cross(e[:, 1], e[:, 2])
    kappa = np.abs(e[:, 0] * c1).sum(axis=1) / np.abs(np.einsum("ei,ei->e", e[:, 0], c1))
    assert kappa[bad].max() < 1e4
