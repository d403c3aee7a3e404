"""Q1 finite elements on the unit cube (oracle side).

Model problem (eq. model, Sec. 2.1): -div(kappa grad u) = f in D, u = u0 on
the boundary, here D = [0,1]^3, u0 = 0, discretised with the C0 Lagrangian
(trilinear, Q1) space on a uniform grid of n^3 hexahedra, h = 1/n (Sec. 2.2
builds the level hierarchy by splitting every cell into 2^3 children).

Conventions (the paper is silent on them):
  node (i, j, k), 0 <= i, j, k <= n, at (i h, j h, k h)
  interior unknown g = (i-1) + (n-1) ((j-1) + (n-1) (k-1)), 1 <= i,j,k <= n-1
  element e = ex + n (ey + n ez), 0 <= ex, ey, ez < n
  local vertex a = ax + 2 ay + 4 az at node (ex+ax, ey+ay, ez+az)

The element stiffness for a per-element constant kappa_e is h kappa_e Khat
with Khat the unit-cube Q1 Laplacian, Khat = k(x)m(x)m + m(x)k(x)m + m(x)m(x)k
for the 1D unit stiffness k = [[1,-1],[-1,1]] and mass m = [[1/3,1/6],[1/6,1/3]].
"""
from __future__ import annotations

import itertools

import numpy as np
import scipy.sparse as sp


def interior_index(n: int, i, j, k):
    return (i - 1) + (n - 1) * ((j - 1) + (n - 1) * (k - 1))


def interior_ijk(n: int) -> np.ndarray:
    """(i, j, k) of every interior unknown in canonical order: int64 [(n-1)^3, 3]."""
    m = n - 1
    g = np.arange(m ** 3)
    return np.stack([g % m + 1, (g // m) % m + 1, g // (m * m) + 1], axis=1)


def element_ijk(n: int) -> np.ndarray:
    e = np.arange(n ** 3)
    return np.stack([e % n, (e // n) % n, e // (n * n)], axis=1)


def local_offsets() -> np.ndarray:
    """Local vertex a -> (ax, ay, az)."""
    return np.array([[a & 1, (a >> 1) & 1, (a >> 2) & 1] for a in range(8)])


def khat() -> np.ndarray:
    """8x8 unit-cube Q1 stiffness by the Kronecker form in the module docstring."""
    k1 = np.array([[1.0, -1.0], [-1.0, 1.0]])
    m1 = np.array([[1.0, 1.0 / 2.0], [1.0 / 2.0, 1.0]]) / 3.0
    # local index a = ax + 2 ay + 4 az  ->  kron order (az, ay, ax)
    return (np.kron(np.kron(m1, m1), k1) + np.kron(np.kron(m1, k1), m1)
            + np.kron(np.kron(k1, m1), m1))


def assemble(n: int, kap: np.ndarray) -> sp.csr_matrix:
    """A_gh = h * sum_{e containing both nodes} kappa_e Khat[a_g(e), a_h(e)].

    One row per interior unknown, neighbour offsets d in {-1,0,1}^3; for each
    entry the shared elements are summed in increasing element index, which
    makes A bitwise symmetric.  Boundary rows/columns are eliminated (u0 = 0).
    """
    kap = np.asarray(kap, dtype=np.float64).reshape(n, n, n)   # [ez, ey, ex]
    K = khat()
    off = local_offsets()
    h = 1.0 / n
    ijk = interior_ijk(n)
    N = ijk.shape[0]
    rows, cols, vals = [], [], []
    for d in itertools.product((-1, 0, 1), repeat=3):
        d = np.array(d)   # (dx, dy, dz)
        nb = ijk + d[None, :]
        ok = np.all((nb >= 1) & (nb <= n - 1), axis=1)
        acc = np.zeros(N)
        # elements containing node p at local a: lower corner p - a; the
        # neighbour p + d is then at local a + d and must be a vertex too.
        # Decreasing local index a = increasing element index.
        for a in range(7, -1, -1):
            b = off[a] + d
            if np.any(b < 0) or np.any(b > 1):
                continue
            lb = b[0] + 2 * b[1] + 4 * b[2]
            corner = ijk - off[a][None, :]
            inside = np.all((corner >= 0) & (corner <= n - 1), axis=1)
            cz = np.clip(corner[:, 2], 0, n - 1)
            cy = np.clip(corner[:, 1], 0, n - 1)
            cx = np.clip(corner[:, 0], 0, n - 1)
            term = kap[cz, cy, cx] * K[a, lb]
            acc = acc + np.where(inside, term, 0.0)
        acc = h * acc
        keep = ok & (acc != 0.0)
        rows.append(np.nonzero(keep)[0])
        cols.append(interior_index(n, nb[keep, 0], nb[keep, 1], nb[keep, 2]))
        vals.append(acc[keep])
    A = sp.csr_matrix((np.concatenate(vals), (np.concatenate(rows), np.concatenate(cols))),
                      shape=(N, N))
    A.sort_indices()
    return A


def load_constant(n: int, f: float = 1.0) -> np.ndarray:
    """b_g = int f phi_g = f h^3 for constant f (each hat integrates to h^3)."""
    return np.full((n - 1) ** 3, f * (1.0 / n) ** 3)


def load_elements(n: int, f_elem: np.ndarray) -> np.ndarray:
    """b_g = int f phi_g for f constant on each element (f_elem[e], element
    layout): each element contributes f_e h^3 / 8 to each of its interior
    corners (a Q1 hat integrates to h^3 / 8 over each of its 8 elements)."""
    f_elem = np.asarray(f_elem, dtype=np.float64)
    eijk = element_ijk(n)
    off = local_offsets()
    w = (1.0 / n) ** 3 / 8.0
    b = np.zeros((n - 1) ** 3)
    for a in range(8):
        p = eijk + off[a][None, :]
        ok = np.all((p >= 1) & (p <= n - 1), axis=1)
        np.add.at(b, interior_index(n, p[ok, 0], p[ok, 1], p[ok, 2]), w * f_elem[ok])
    return b


GAUSS3_X = np.array([-np.sqrt(3.0 / 5.0), 0.0, np.sqrt(3.0 / 5.0)])
GAUSS3_W = np.array([5.0 / 9.0, 8.0 / 9.0, 5.0 / 9.0])


def _gauss_points(n: int):
    """Per element: 27 points (global coords) and weights, as [n^3, 27, 3], [27]."""
    h = 1.0 / n
    t = 0.5 * (GAUSS3_X + 1.0)
    pts = np.array(list(itertools.product(t, t, t)))[:, ::-1]   # (x, y, z), x fastest
    w = np.array([a * b * c for a, b, c in itertools.product(GAUSS3_W, GAUSS3_W, GAUSS3_W)]) / 8.0
    eijk = element_ijk(n)
    X = (eijk[:, None, :] + pts[None, :, :]) * h
    return X, pts, w * h ** 3


def _shape(pts: np.ndarray) -> np.ndarray:
    """Trilinear shape functions at reference points [27, 3] -> [27, 8]."""
    off = local_offsets()
    return np.prod(np.where(off[None, :, :] == 1, pts[:, None, :], 1.0 - pts[:, None, :]), axis=2)


def load_function(n: int, f) -> np.ndarray:
    """b_g = sum_e int_e f N_a by 3x3x3 Gauss (used for manufactured solutions)."""
    X, pts, w = _gauss_points(n)
    N = _shape(pts)
    fx = f(X[..., 0], X[..., 1], X[..., 2])                 # [E, 27]
    be = np.einsum("eq,q,qa->ea", fx, w, N)                 # [E, 8]
    eijk = element_ijk(n)
    off = local_offsets()
    b = np.zeros((n - 1) ** 3)
    for a in range(8):
        p = eijk + off[a][None, :]
        ok = np.all((p >= 1) & (p <= n - 1), axis=1)
        np.add.at(b, interior_index(n, p[ok, 0], p[ok, 1], p[ok, 2]), be[ok, a])
    return b


def l2_error(n: int, u: np.ndarray, exact) -> float:
    """|| u_h - exact ||_L2 by 3x3x3 Gauss on every element."""
    X, pts, w = _gauss_points(n)
    N = _shape(pts)
    full = np.zeros((n + 1, n + 1, n + 1))
    ijk = interior_ijk(n)
    full[ijk[:, 2], ijk[:, 1], ijk[:, 0]] = u
    eijk = element_ijk(n)
    off = local_offsets()
    ue = np.stack([full[eijk[:, 2] + off[a, 2], eijk[:, 1] + off[a, 1], eijk[:, 0] + off[a, 0]]
                   for a in range(8)], axis=1)              # [E, 8]
    uh = ue @ N.T                                           # [E, 27]
    ex = exact(X[..., 0], X[..., 1], X[..., 2])
    return float(np.sqrt(np.sum((uh - ex) ** 2 * w[None, :])))


def qoi_weights(n: int, qoi: int) -> np.ndarray:
    """w with Q(u_h) = w . u for interior u (eq. model's QoI, Sec. 2.1).

    qoi 0: domain average, int_D u_h / |D| = h^3 sum_g u_g (each interior
           node touches 8 elements, each contributing h^3/8).
    qoi 1: average over S = [1/4, 3/4]^3: (1/|S|) sum_{e in S} (h^3/8) sum_a u_{e,a}
           = h^3 * sum_g c_g u_g / (8 |S|) * 8, c_g = number of elements of S at g.
    The trilinear integral over a cube is its volume times the vertex mean.
    """
    h = 1.0 / n
    if qoi == 0:
        return np.full((n - 1) ** 3, h ** 3)
    if n % 4:
        raise ValueError("subcube QoI needs n divisible by 4")
    eijk = element_ijk(n)
    inS = np.all((eijk >= n // 4) & (eijk < 3 * n // 4), axis=1)
    cnt = np.zeros((n + 1, n + 1, n + 1))
    off = local_offsets()
    for a in range(8):
        p = eijk[inS] + off[a][None, :]
        np.add.at(cnt, (p[:, 2], p[:, 1], p[:, 0]), 1.0)
    ijk = interior_ijk(n)
    c = cnt[ijk[:, 2], ijk[:, 1], ijk[:, 0]]
    vol = 0.125
    return c * (h ** 3 / 8.0) / vol
