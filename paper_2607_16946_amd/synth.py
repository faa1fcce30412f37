"""Seeded synthetic workloads shaped like the paper's (shared by tests, bench and oracle checks).

This module holds no arithmetic of the method: it produces oriented points,
per-point height-polynomial coefficients and query points.  Coefficients are
analytic (there is no trained network): for a primitive with implicit function
F (F < 0 inside) and outward normal n = grad F / |grad F|, the height function
over the tangent plane is Q(s,t) = -1/2 (s,t) Hess_tan F (s,t)^T / |grad F| to
second order, so

    a20 = -1/2 s^T H s / |grad F|,  a02 = -1/2 t^T H t / |grad F|,
    a11 = -s^T H t / |grad F|,      a00 = a10 = a01 = 0,

written in the per-point tangent frame (s, t) that the library's input format
fixes: e = x-hat if |n_x| < 0.9 else y-hat, s = normalize(e - <e,n> n),
t = n x s.  Coefficient order everywhere is (a00, a01, a10, a11, a02, a20).

Workload shapes follow the paper: a 4096-point cloud (Fig. 1), a 128^3
evaluation grid (Fig. 6), million-point noisy scans with outliers (Sec. 5.2,
5.3), sphere tracing (Sec. 5.3).  Seeds: PCG64(20260703 + k) for workload k,
PCG64(40000 + j) for serving cloud j.
"""

from __future__ import annotations

import dataclasses
import math

import numpy as np

SEED_BASE = 20260703
SERVE_SEED_BASE = 40000


def rng_for(k: int) -> np.random.Generator:
    return np.random.Generator(np.random.PCG64(SEED_BASE + k))


@dataclasses.dataclass
class Cloud:
    p: np.ndarray          # [N,3] float32 positions
    n: np.ndarray          # [N,3] float32 unit normals
    a: np.ndarray          # [N,6] float32 coefficients (a00, a01, a10, a11, a02, a20)
    meta: dict

    @property
    def N(self) -> int:
        return self.p.shape[0]


# ---------------------------------------------------------------------------
# Input-frame convention and analytic coefficients
# ---------------------------------------------------------------------------

def tangent_frame(n: np.ndarray):
    """Per-point (s, t) of the input format, for unit normals n [N,3] (float64)."""
    n = np.asarray(n, dtype=np.float64)
    e = np.zeros_like(n)
    use_x = np.abs(n[:, 0]) < 0.9
    e[use_x, 0] = 1.0
    e[~use_x, 1] = 1.0
    s = e - np.sum(e * n, axis=1, keepdims=True) * n
    s /= np.linalg.norm(s, axis=1, keepdims=True)
    t = np.cross(n, s)
    return s, t


def coeffs_from_implicit(grad: np.ndarray, hess: np.ndarray):
    """Unit normals and (a00..a20) from grad F [N,3] and Hess F [N,3,3] at surface points."""
    g = np.linalg.norm(grad, axis=1)
    n = grad / g[:, None]
    s, t = tangent_frame(n)
    Hs = np.einsum("nij,nj->ni", hess, s)
    Ht = np.einsum("nij,nj->ni", hess, t)
    a = np.zeros((n.shape[0], 6))
    a[:, 5] = -0.5 * np.sum(s * Hs, axis=1) / g   # a20
    a[:, 4] = -0.5 * np.sum(t * Ht, axis=1) / g   # a02
    a[:, 3] = -np.sum(s * Ht, axis=1) / g          # a11
    return n, a


def random_rotation(rng: np.random.Generator) -> np.ndarray:
    q = rng.normal(size=4)
    q /= np.linalg.norm(q)
    w, x, y, z = q
    return np.array([
        [1 - 2 * (y * y + z * z), 2 * (x * y - z * w), 2 * (x * z + y * w)],
        [2 * (x * y + z * w), 1 - 2 * (x * x + z * z), 2 * (y * z - x * w)],
        [2 * (x * z - y * w), 2 * (y * z + x * w), 1 - 2 * (x * x + y * y)],
    ])


# ---------------------------------------------------------------------------
# Primitives: implicit function, derivatives, area-uniform sampling
# ---------------------------------------------------------------------------

class Ellipsoid:
    def __init__(self, center, rot, axes):
        self.c = np.asarray(center, dtype=np.float64)
        self.Rm = np.asarray(rot, dtype=np.float64)      # columns: local axes in world
        self.ax = np.asarray(axes, dtype=np.float64)

    def local(self, x):
        return (x - self.c) @ self.Rm

    def F(self, x):
        y = self.local(x)
        return np.sum((y / self.ax) ** 2, axis=1) - 1.0

    def grad_hess(self, x):
        y = self.local(x)
        gl = 2.0 * y / self.ax ** 2
        grad = gl @ self.Rm.T
        Hl = np.diag(2.0 / self.ax ** 2)
        hess = np.broadcast_to(self.Rm @ Hl @ self.Rm.T, (x.shape[0], 3, 3)).copy()
        return grad, hess

    def area(self, rng) -> float:
        u = rng.normal(size=(20000, 3))
        u /= np.linalg.norm(u, axis=1, keepdims=True)
        f = np.prod(self.ax) * np.sqrt(np.sum((u / self.ax) ** 2, axis=1))
        return float(4.0 * math.pi * f.mean())

    def sample(self, rng, m: int):
        out = []
        got = 0
        while got < m:
            u = rng.normal(size=(2 * m + 16, 3))
            u /= np.linalg.norm(u, axis=1, keepdims=True)
            acc = self.ax.min() * np.sqrt(np.sum((u / self.ax) ** 2, axis=1))
            keep = rng.uniform(size=u.shape[0]) < acc
            y = u[keep] * self.ax
            out.append(y)
            got += y.shape[0]
        y = np.concatenate(out)[:m]
        return y @ self.Rm.T + self.c


class RingTorus:
    def __init__(self, center, rot, R, r):
        self.c = np.asarray(center, dtype=np.float64)
        self.Rm = np.asarray(rot, dtype=np.float64)
        self.R = float(R)
        self.r = float(r)

    def local(self, x):
        return (x - self.c) @ self.Rm

    def F(self, x):
        y = self.local(x)
        rho = np.sqrt(y[:, 0] ** 2 + y[:, 1] ** 2)
        return (rho - self.R) ** 2 + y[:, 2] ** 2 - self.r ** 2

    def grad_hess(self, x):
        y = self.local(x)
        X, Y, Z = y[:, 0], y[:, 1], y[:, 2]
        rho = np.sqrt(X * X + Y * Y)
        e = rho - self.R
        gl = np.stack([2 * e * X / rho, 2 * e * Y / rho, 2 * Z], axis=1)
        Hl = np.zeros((x.shape[0], 3, 3))
        Hl[:, 0, 0] = 2 * X * X / rho ** 2 + 2 * e * Y * Y / rho ** 3
        Hl[:, 1, 1] = 2 * Y * Y / rho ** 2 + 2 * e * X * X / rho ** 3
        Hl[:, 0, 1] = Hl[:, 1, 0] = 2 * X * Y / rho ** 2 - 2 * e * X * Y / rho ** 3
        Hl[:, 2, 2] = 2.0
        grad = gl @ self.Rm.T
        hess = np.einsum("ij,njk,lk->nil", self.Rm, Hl, self.Rm)
        return grad, hess

    def area(self, rng) -> float:
        return 4.0 * math.pi ** 2 * self.R * self.r

    def surface_point(self, theta, psi):
        rr = self.R + self.r * np.cos(theta)
        y = np.stack([rr * np.cos(psi), rr * np.sin(psi), self.r * np.sin(theta)], axis=1)
        return y @ self.Rm.T + self.c

    def sample(self, rng, m: int):
        out = []
        got = 0
        while got < m:
            k = 2 * m + 16
            th = rng.uniform(0, 2 * math.pi, size=k)
            ps = rng.uniform(0, 2 * math.pi, size=k)
            keep = rng.uniform(size=k) < (self.R + self.r * np.cos(th)) / (self.R + self.r)
            out.append(self.surface_point(th[keep], ps[keep]))
            got += int(keep.sum())
        return np.concatenate(out)[:m]


def random_primitives(rng, count: int):
    prims = []
    for _ in range(count):
        c = rng.uniform(-0.6, 0.6, size=3)
        Rm = random_rotation(rng)
        if rng.uniform() < 0.5:
            prims.append(Ellipsoid(c, Rm, rng.uniform(0.1, 0.5, size=3)))
        else:
            R = rng.uniform(0.2, 0.5)
            prims.append(RingTorus(c, Rm, R, rng.uniform(0.1, 0.6 * R)))
    return prims


def sample_union(rng, prims, N: int, density=None):
    """Area-uniform samples on the boundary of the union of primitives.

    Samples inside any other primitive are dropped.  ``density(x) in (0, 1]``
    optionally thins the samples (acceptance probability).  Returns clean
    points, unit normals and analytic coefficients."""
    areas = np.array([pr.area(rng) for pr in prims])
    probs = areas / areas.sum()
    P, Nn, A = [], [], []
    got = 0
    while got < N:
        batch = max(4096, 2 * (N - got))
        counts = rng.multinomial(batch, probs)
        for j, (pr, m) in enumerate(zip(prims, counts)):
            if m == 0:
                continue
            x = pr.sample(rng, int(m))
            keep = np.ones(x.shape[0], dtype=bool)
            for k, other in enumerate(prims):
                if k != j:
                    keep &= other.F(x) >= 0.0
            if density is not None:
                keep &= rng.uniform(size=x.shape[0]) < density(x)
            x = x[keep]
            if x.shape[0] == 0:
                continue
            grad, hess = pr.grad_hess(x)
            n, a = coeffs_from_implicit(grad, hess)
            P.append(x)
            Nn.append(n)
            A.append(a)
            got += x.shape[0]
    P = np.concatenate(P)
    Nn = np.concatenate(Nn)
    A = np.concatenate(A)
    perm = rng.permutation(P.shape[0])[:N]
    return P[perm], Nn[perm], A[perm]


def padded_bbox(p: np.ndarray, pad: float = 0.1):
    lo = p.min(axis=0).astype(np.float64)
    hi = p.max(axis=0).astype(np.float64)
    ext = hi - lo
    return lo - pad * ext, hi + pad * ext


def lattice(lo, hi, res: int) -> np.ndarray:
    axes = [np.linspace(lo[k], hi[k], res) for k in range(3)]
    g = np.stack(np.meshgrid(*axes, indexing="ij"), axis=-1).reshape(-1, 3)
    return g.astype(np.float32)


def _f32(*arrs):
    return tuple(np.ascontiguousarray(np.asarray(a, dtype=np.float32)) for a in arrs)


# ---------------------------------------------------------------------------
# Workloads
# ---------------------------------------------------------------------------

def sphere_cloud(N: int = 4096, seed: int = SEED_BASE + 1, jitter: float = 0.01, radius: float = 1.0) -> Cloud:
    """Points uniform on a sphere, exact outward normals, principal curvatures
    -(1+eps)/radius per direction with eps ~ N(0, jitter^2), zero shift."""
    rng = np.random.Generator(np.random.PCG64(seed))
    z = rng.normal(size=(N, 3))
    n = z / np.linalg.norm(z, axis=1, keepdims=True)
    p = radius * n
    k = -(1.0 + jitter * rng.normal(size=(N, 2))) / radius
    a = np.zeros((N, 6))
    a[:, 5] = 0.5 * k[:, 0]
    a[:, 4] = 0.5 * k[:, 1]
    p, n, a = _f32(p, n, a)
    return Cloud(p, n, a, {"shape": "sphere", "seed": seed, "radius": radius, "jitter": jitter})


def torus_cloud(N: int, R: float = 0.6, r: float = 0.25, seed: int = SEED_BASE + 7, noise: float = 0.0):
    """N points uniform (by area) on one ring torus with a random orientation,
    exact normals and analytic coefficients.  Returns (cloud, the RingTorus)."""
    rng = np.random.Generator(np.random.PCG64(seed))
    prim = RingTorus(np.zeros(3), random_rotation(rng), R, r)
    p, n, a = sample_union(rng, [prim], N)
    p = p + rng.normal(scale=noise, size=p.shape)
    p, n, a = _f32(p, n, a)
    return Cloud(p, n, a, {"shape": "ring torus", "R": R, "r": r, "seed": seed, "noise": noise}), prim


def cap_cloud(N: int = 1400, Q: int = 1500, radius: float = 50.0, seed: int = SEED_BASE + 11):
    """A nearly flat cloud: N points on the cap |xy| < 1 of a sphere of the given
    radius (center (0, 0, -radius)), outward normals, and curvatures
    -(1 +- e)/radius with e ~ U(0.15, 0.3) along s and t (unequal, so no point
    is umbilic).  Half of the Q queries lie within 0.1 of the cap along the
    normal, half uniform in its bbox padded by 0.2.  Returns (cloud, queries)."""
    rng = np.random.Generator(np.random.PCG64(seed))
    xy = rng.uniform(-1.0, 1.0, size=(4 * N, 2))
    xy = xy[np.hypot(xy[:, 0], xy[:, 1]) < 1.0][:N]
    z = np.sqrt(radius ** 2 - (xy ** 2).sum(axis=1)) - radius
    p = np.c_[xy, z]
    n = (p - np.array([0.0, 0.0, -radius])) / radius
    e = rng.uniform(0.15, 0.3, size=len(p))
    a = np.zeros((len(p), 6))
    a[:, 4] = -0.5 / radius * (1.0 + e)     # a02
    a[:, 5] = -0.5 / radius * (1.0 - e)     # a20
    k = rng.integers(len(p), size=Q // 2)
    near = p[k] + n[k] * rng.uniform(-0.1, 0.1, size=(Q // 2, 1))
    box = rng.uniform(p.min(axis=0) - 0.2, p.max(axis=0) + 0.2, size=(Q - Q // 2, 3))
    p, n, a, x = _f32(p, n, a, np.r_[near, box])
    return Cloud(p, n, a, {"shape": "spherical cap", "radius": radius, "seed": seed}), x


def mixed_forms_cloud(N: int = 6000, seed: int = 21) -> Cloud:
    """The mid cloud's points with general coefficients interleaved in input
    order: shift a00, tilt a10/a01, both, nearly flat points (a02, a20 scaled
    by 1e-4: large radii) and exactly flat ones (a11 = a02 = a20 = 0: both
    curvatures at the floor), next to the analytic ones."""
    cl, _ = mid(N=N, grid=4)
    rng = np.random.default_rng(seed)
    a = cl.a.astype(np.float64).copy()
    kind = rng.integers(0, 6, size=N)
    a[kind == 1, 0] = rng.normal(0, 0.01, size=(kind == 1).sum())                 # shift
    a[kind == 2, 1:3] = rng.normal(0, 0.2, size=((kind == 2).sum(), 2))          # tilt
    both = kind == 3
    a[both, 0] = rng.normal(0, 0.01, size=both.sum())
    a[both, 1:3] = rng.normal(0, 0.2, size=(both.sum(), 2))
    a[kind == 4, 4:6] *= 1e-4                                                     # nearly flat: large L
    a[kind == 5, 3:6] = 0.0                                                       # flat
    return Cloud(cl.p, cl.n, a.astype(np.float32), {"shape": "mixed forms", "seed": seed})


def tiny(Q: int = 4096, N: int = 4096):
    """Plain method, tiny: N points on the unit sphere, Q queries uniform in [-1.5,1.5]^3."""
    cl = sphere_cloud(N, SEED_BASE + 1)
    rng = rng_for(101)
    x = rng.uniform(-1.5, 1.5, size=(Q, 3)).astype(np.float32)
    return cl, x


def primitives_cloud(N: int, nprim: int, noise: float, seed: int, density=None, outlier_frac: float = 0.0):
    rng = np.random.Generator(np.random.PCG64(seed))
    prims = random_primitives(rng, nprim)
    dens = None
    if density is not None:
        kvec = rng.normal(size=3) * density
        dens = lambda x: 0.1 + 0.9 * 0.5 * (1.0 + np.sin(x @ kvec))  # noqa: E731
    n_out = int(round(outlier_frac * N))
    n_in = N - n_out
    p, n, a = sample_union(rng, prims, n_in, dens)
    p = p + rng.normal(scale=noise, size=p.shape)
    meta = {"nprim": nprim, "noise": noise, "seed": seed,
            "prims": [type(pr).__name__ for pr in prims]}
    if n_out > 0:
        lo, hi = p.min(axis=0), p.max(axis=0)
        area = sum(pr.area(rng) for pr in prims)
        ell = math.sqrt(area / n_in)
        po = rng.uniform(lo, hi, size=(n_out, 3))
        no = rng.normal(size=(n_out, 3))
        no /= np.linalg.norm(no, axis=1, keepdims=True)
        ao = np.zeros((n_out, 6))
        ao[:, 4] = ao[:, 5] = -0.5 / ell
        p = np.concatenate([p, po])
        n = np.concatenate([n, no])
        a = np.concatenate([a, ao])
        perm = rng.permutation(N)
        p, n, a = p[perm], n[perm], a[perm]
        meta["outliers"] = n_out
        meta["spacing"] = ell
    p, n, a = _f32(p, n, a)
    return Cloud(p, n, a, meta), prims


def mid(N: int = 131072, grid: int = 128):
    """Plain method, mid: union of 8 random ellipsoids / ring tori, sigma=0.002
    position noise, queries on a grid^3 lattice over the bbox padded 10%."""
    cl, _ = primitives_cloud(N, 8, 0.002, SEED_BASE + 2)
    lo, hi = padded_bbox(cl.p, 0.1)
    x = lattice(lo, hi, grid)
    cl.meta["grid"] = grid
    return cl, x


def diff_workload(N: int = 32768, Q: int = 1 << 20):
    """Differentiation: one ellipsoid; half the queries within 0.05 of the
    surface along the normal, half uniform in the padded bbox.  Returns the
    cloud, the queries and the loss mask (near-surface half)."""
    rng = rng_for(3)
    ell = Ellipsoid(np.zeros(3), random_rotation(rng), rng.uniform(0.1, 0.5, size=3))
    x = ell.sample(rng, N)
    grad, hess = ell.grad_hess(x)
    n, a = coeffs_from_implicit(grad, hess)
    p, n32, a32 = _f32(x, n, a)
    cl = Cloud(p, n32, a32, {"shape": "ellipsoid", "axes": ell.ax.tolist()})
    qn = Q // 2
    xs = ell.sample(rng, qn)
    gs, _ = ell.grad_hess(xs)
    ns = gs / np.linalg.norm(gs, axis=1, keepdims=True)
    near = xs + rng.uniform(-0.05, 0.05, size=(qn, 1)) * ns
    lo, hi = padded_bbox(p, 0.1)
    far = rng.uniform(lo, hi, size=(Q - qn, 3))
    q = np.concatenate([near, far]).astype(np.float32)
    mask = np.zeros(Q, dtype=bool)
    mask[:qn] = True
    return cl, q, mask


def serving_cloud(j: int, nmin: int = 1024, nmax: int = 262144) -> Cloud:
    """Serving cloud j: N log-uniform in [nmin, nmax], sphere generator of the tiny workload."""
    rng = np.random.Generator(np.random.PCG64(SERVE_SEED_BASE + j))
    N = int(round(math.exp(rng.uniform(math.log(nmin), math.log(nmax)))))
    return sphere_cloud(N, SERVE_SEED_BASE + 1000 + j)


def large(N: int = 1 << 20, Q: int = 1 << 20):
    """Large photogrammetry-like: 32 primitives, density varying 10x, sigma=0.005,
    3% outliers with random normals; Q uniform queries in the padded bbox."""
    cl, _ = primitives_cloud(N, 32, 0.005, SEED_BASE + 5, density=6.0, outlier_frac=0.03)
    rng = rng_for(105)
    lo, hi = padded_bbox(cl.p, 0.1)
    x = rng.uniform(lo, hi, size=(Q, 3)).astype(np.float32)
    return cl, x


def camera_rays(res: int, radius: float = 3.0, fov_deg: float = 45.0, seed: int = 0,
                target=(0.0, 0.0, 0.0)):
    """Pinhole camera on a sphere of given radius aimed at target; res x res rays."""
    rng = np.random.Generator(np.random.PCG64(SEED_BASE + 900 + seed))
    d = rng.normal(size=3)
    d /= np.linalg.norm(d)
    eye = np.asarray(target) + radius * d
    fwd = np.asarray(target) - eye
    fwd /= np.linalg.norm(fwd)
    up0 = np.array([0.0, 0.0, 1.0]) if abs(fwd[2]) < 0.9 else np.array([1.0, 0.0, 0.0])
    right = np.cross(fwd, up0)
    right /= np.linalg.norm(right)
    up = np.cross(right, fwd)
    h = math.tan(math.radians(fov_deg) / 2)
    u = (np.arange(res) + 0.5) / res * 2 - 1
    uu, vv = np.meshgrid(u, u, indexing="xy")
    dirs = fwd[None] + h * (uu.reshape(-1, 1) * right[None] + vv.reshape(-1, 1) * up[None])
    dirs /= np.linalg.norm(dirs, axis=1, keepdims=True)
    org = np.broadcast_to(eye, dirs.shape).copy()
    return org.astype(np.float32), dirs.astype(np.float32)
