"""Seeded synthetic inputs for the DEC multigrid workloads.

This module is shared by the FP64 reference (``oracle/``) and by the HIP path.  It holds
random draws and closed-form test functions evaluated at given coordinates, and nothing of
the method itself: no subdivision, no DEC operator, no smoothing, no solve.  Vertex
coordinates of the subdivided workloads are always passed in by the caller, each side passing
its own.  The one exception is the input of the non-nested workload: meshes and the geometric
maps between them are what a user hands to the method, so they are generated here
(``jittered_grid``, ``grid_point_location``) and given to both sides alike.

Workloads (unit square meshes are 2-D right-triangle grids, spheres are icospheres):

* ``c1``: 4x4 cells, 4 subdivisions, f = 2 pi^2 sin(pi x) sin(pi y) (the Poisson check of
  Sec. 3.1 with a manufactured solution).
* ``c2``: icosahedron, 7 projected subdivisions, f = sum of real spherical harmonics of
  degree 1..8 with N(0,1) coefficients (seed 2).
* ``c3``: 8x8 cells, 8 subdivisions (2049 x 2049 vertices), f ~ N(0,1) per vertex (seed 3).
* ``c4``: 256 instances, a seeded mix of icosphere levels 4..7 and square grids 33^2..513^2.
* ``c5``: porous convection on 4x4 cells, 6 subdivisions (257 x 257): white noise for the
  log-permeability (seed 5), temperature noise (seed 6), loss weights (seed 7).
"""
from __future__ import annotations

import math

import numpy as np

SEED_C2 = 2
SEED_C3 = 3
SEED_C4 = 4
SEED_C5_G = 5
SEED_C5_T = 6
SEED_C5_W = 7

# (base cells per side, subdivisions) for each square workload; spheres give the level.
C1 = dict(base_cells=4, nsub=4)
C2 = dict(sphere_level=7)
C3 = dict(base_cells=8, nsub=8)
# the largest V-cycle sweep mesh: the 32-triangle square, 4 cubic subdivisions (325 x 325)
E1_CUBIC = dict(base_cells=4, nsub=4, cubic_mask=0b1111)
SEED_E1 = 8
C5 = dict(base_cells=4, nsub=6, Ra=1000.0, phi=0.1, steps=200, ckpt=20, noise=1e-2,
          g_smooth_sweeps=20, g_smooth_omega=0.8)

# The C4 menu: ("sphere", level) or ("square", vertices-per-side).  Squares use a 4x4-cell
# base; vertices-per-side 33..513 are 3..7 subdivisions of it.
C4_MENU = [("sphere", 4), ("sphere", 5), ("sphere", 6), ("sphere", 7),
           ("square", 33), ("square", 65), ("square", 129), ("square", 257), ("square", 513)]


def normal(n: int, seed: int) -> np.ndarray:
    """i.i.d. N(0,1) draws, float64, from numpy's PCG64 ``default_rng(seed)``."""
    return np.random.default_rng(seed).standard_normal(int(n))


def uniform01(n: int, seed: int) -> np.ndarray:
    """i.i.d. U[0,1) draws, float64 (the consistent-RHS trick b = L r of Sec. 3.1)."""
    return np.random.default_rng(seed).random(int(n))


def manufactured_c1(xyz: np.ndarray) -> np.ndarray:
    """f = 2 pi^2 sin(pi x) sin(pi y); u = sin(pi x) sin(pi y) solves -lap u = f, u = 0 on the
    boundary of the unit square."""
    x, y = xyz[:, 0], xyz[:, 1]
    return 2.0 * math.pi ** 2 * np.sin(math.pi * x) * np.sin(math.pi * y)


def manufactured_c1_solution(xyz: np.ndarray) -> np.ndarray:
    x, y = xyz[:, 0], xyz[:, 1]
    return np.sin(math.pi * x) * np.sin(math.pi * y)


# ---------------------------------------------------------------- spherical harmonics
def _assoc_legendre(lmax: int, x: np.ndarray) -> dict:
    """P_l^m(x) for 0 <= m <= l <= lmax without the Condon-Shortley phase, by the standard
    three-term recurrences (m-diagonal, then upward in l)."""
    P = {}
    s = np.sqrt(np.maximum(0.0, 1.0 - x * x))
    pmm = np.ones_like(x)
    for m in range(lmax + 1):
        if m > 0:
            pmm = pmm * (2 * m - 1) * s
        P[(m, m)] = pmm
        if m + 1 <= lmax:
            P[(m + 1, m)] = x * (2 * m + 1) * pmm
        for l in range(m + 2, lmax + 1):
            P[(l, m)] = ((2 * l - 1) * x * P[(l - 1, m)] - (l + m - 1) * P[(l - 2, m)]) / (l - m)
    return P


def real_sph_harm(lmax: int, xyz: np.ndarray) -> dict:
    """Orthonormal real spherical harmonics Y_lm on the unit sphere, 0 <= l <= lmax,
    -l <= m <= l: sqrt(2) N P_l^|m| cos(m phi) for m > 0, N P_l^0 for m = 0 and
    sqrt(2) N P_l^|m| sin(|m| phi) for m < 0, N = sqrt((2l+1)/(4 pi) (l-|m|)!/(l+|m|)!).
    Points are projected to the unit sphere first."""
    r = np.sqrt(xyz[:, 0] ** 2 + xyz[:, 1] ** 2 + xyz[:, 2] ** 2)
    ct = xyz[:, 2] / r
    ph = np.arctan2(xyz[:, 1], xyz[:, 0])
    P = _assoc_legendre(lmax, ct)
    Y = {}
    for l in range(lmax + 1):
        for m in range(-l, l + 1):
            am = abs(m)
            N = math.sqrt((2 * l + 1) / (4 * math.pi) * math.factorial(l - am) / math.factorial(l + am))
            if m == 0:
                Y[(l, m)] = N * P[(l, 0)]
            elif m > 0:
                Y[(l, m)] = math.sqrt(2.0) * N * P[(l, am)] * np.cos(am * ph)
            else:
                Y[(l, m)] = math.sqrt(2.0) * N * P[(l, am)] * np.sin(am * ph)
    return Y


def sh_coefficients(seed: int = SEED_C2, lmax: int = 8) -> list:
    """[(l, m, c_lm)] with c_lm ~ N(0,1) drawn in the order l = 1..lmax, m = -l..l."""
    c = normal((lmax + 1) ** 2 - 1, seed)
    out, k = [], 0
    for l in range(1, lmax + 1):
        for m in range(-l, l + 1):
            out.append((l, m, float(c[k])))
            k += 1
    return out


def sphere_rhs(xyz: np.ndarray, coeffs: list) -> np.ndarray:
    """f = sum c_lm Y_lm evaluated at the vertices (zero mean over the continuous sphere)."""
    lmax = max(l for l, _, _ in coeffs)
    Y = real_sph_harm(lmax, xyz)
    f = np.zeros(len(xyz))
    for l, m, c in coeffs:
        f += c * Y[(l, m)]
    return f


def sphere_exact(xyz: np.ndarray, coeffs: list) -> np.ndarray:
    """Continuous zero-mean solution of -lap_S u = f: u = sum c_lm Y_lm / (l (l+1))."""
    lmax = max(l for l, _, _ in coeffs)
    Y = real_sph_harm(lmax, xyz)
    u = np.zeros(len(xyz))
    for l, m, c in coeffs:
        u += c / (l * (l + 1)) * Y[(l, m)]
    return u


# ---------------------------------------------------------------- batched mix
def c4_instances(seed: int = SEED_C4, n: int = 256) -> list:
    """The seeded C4 mix: a list of dicts {kind, level|side, nsub, rhs_seed}."""
    types = np.random.default_rng(seed).integers(0, len(C4_MENU), n)
    out = []
    for i, t in enumerate(types):
        kind, v = C4_MENU[int(t)]
        if kind == "sphere":
            out.append(dict(kind="sphere", nsub=v, rhs_seed=4000 + i))
        else:
            nsub = int(round(math.log2((v - 1) / 4)))
            out.append(dict(kind="square", base_cells=4, nsub=nsub, rhs_seed=4000 + i))
    return out


# ---------------------------------------------------------------- porous convection
def c5_logk_noise(nv: int) -> np.ndarray:
    """White noise for the log-permeability field g before smoothing (seed 5)."""
    return normal(nv, SEED_C5_G)


def c5_initial_temperature(xyz: np.ndarray) -> np.ndarray:
    """T0 = 1 - y + noise * N(0,1) (seed 6).  Noise is drawn for every vertex; the walls
    y = 0 and y = 1 are reset to 1 and 0 exactly, so they hold their conductive values."""
    y = xyz[:, 1]
    T = 1.0 - y + C5["noise"] * normal(len(xyz), SEED_C5_T)
    T[y == 0.0] = 1.0
    T[y == 1.0] = 0.0
    return T


def c5_loss_weights(nv: int) -> np.ndarray:
    """Loss J = sum_i w_i T_i(final) with w ~ N(0,1) (seed 7)."""
    return normal(nv, SEED_C5_W)


# ---------------------------------------------------------------- non-nested map workload
SEED_MAPS = 9
MAPS_CELLS = (4, 8, 16, 32, 64)   # cells per side, coarsest first
MAPS_AMP = 0.15                   # interior vertex jitter, in cell widths


def jittered_grid(n: int, seed: int, amp: float = MAPS_AMP):
    """Input mesh of the non-nested workload: the unit square with n x n cells split along the
    SW-NE diagonal, every interior vertex moved by U[-amp, amp] / n in x and in y (seeded).
    Vertex (i, j) is j (n+1) + i; cell (ci, cj) gives triangles 2 (cj n + ci) and +1."""
    j, i = np.mgrid[0:n + 1, 0:n + 1]
    xyz = np.zeros(((n + 1) ** 2, 3))
    xyz[:, 0] = i.ravel() / n
    xyz[:, 1] = j.ravel() / n
    inner = ((i > 0) & (i < n) & (j > 0) & (j < n)).ravel()
    d = np.random.default_rng(seed).uniform(-amp, amp, size=(int(inner.sum()), 2)) / n
    xyz[inner, :2] += d
    a = (np.arange(n)[None, :] + (n + 1) * np.arange(n)[:, None]).ravel()
    tri = np.empty((2 * n * n, 3), dtype=np.int32)
    tri[0::2] = np.column_stack([a, a + 1, a + n + 2])
    tri[1::2] = np.column_stack([a, a + n + 2, a + n + 1])
    e1 = xyz[tri[:, 1], :2] - xyz[tri[:, 0], :2]
    e2 = xyz[tri[:, 2], :2] - xyz[tri[:, 0], :2]
    assert np.all(e1[:, 0] * e2[:, 1] - e1[:, 1] * e2[:, 0] > 0), "jitter inverted a triangle"
    return xyz, tri


def grid_point_location(xyz_c, tri_c, n_c: int, xyz_f, drop: float = 1e-14):
    """The geometric map sending every fine vertex to the same point of the coarse jittered
    grid: M(f) (coarse x fine, scipy CSC) with column j the barycentric coordinates of fine
    vertex j in the coarse triangle that holds it.  Candidates are the triangles of the 3 x 3
    cells around the point's cell (vertices move by less than half a cell); the one whose
    smallest coordinate is largest wins.  Coordinates at or below `drop` are removed, so points
    on coarse edges or at coarse vertices name that edge or vertex."""
    import scipy.sparse as sp
    p = np.asarray(xyz_f)[:, :2]
    nf = len(p)
    cell = np.clip(np.floor(p * n_c).astype(np.int64), 0, n_c - 1)
    best = np.full(nf, -np.inf)
    lam = np.zeros((nf, 3))
    which = np.zeros(nf, dtype=np.int64)
    for dj in (-1, 0, 1):
        for di in (-1, 0, 1):
            ci = cell[:, 0] + di
            cj = cell[:, 1] + dj
            ok = (ci >= 0) & (ci < n_c) & (cj >= 0) & (cj < n_c)
            for s in (0, 1):
                t = np.where(ok, 2 * (np.clip(cj, 0, n_c - 1) * n_c + np.clip(ci, 0, n_c - 1)) + s, 0)
                A = xyz_c[tri_c[t, 0], :2]
                B = xyz_c[tri_c[t, 1], :2]
                C = xyz_c[tri_c[t, 2], :2]
                den = (B[:, 0] - A[:, 0]) * (C[:, 1] - A[:, 1]) - (B[:, 1] - A[:, 1]) * (C[:, 0] - A[:, 0])
                lb = ((p[:, 0] - A[:, 0]) * (C[:, 1] - A[:, 1]) - (p[:, 1] - A[:, 1]) * (C[:, 0] - A[:, 0])) / den
                lc = ((B[:, 0] - A[:, 0]) * (p[:, 1] - A[:, 1]) - (B[:, 1] - A[:, 1]) * (p[:, 0] - A[:, 0])) / den
                la = 1.0 - lb - lc
                m = np.minimum(np.minimum(la, lb), lc)
                m = np.where(ok, m, -np.inf)
                take = m > best
                best = np.where(take, m, best)
                lam[take] = np.column_stack([la, lb, lc])[take]
                which[take] = t[take]
    assert best.min() >= -1e-12, "a fine vertex lies outside the coarse mesh"
    rows, cols, vals = [], [], []
    for q in range(3):
        keep = lam[:, q] > drop
        rows.append(tri_c[which[keep], q])
        cols.append(np.nonzero(keep)[0])
        vals.append(lam[keep, q])
    M = sp.csc_matrix((np.concatenate(vals), (np.concatenate(rows), np.concatenate(cols))),
                      shape=(len(xyz_c), nf))
    M.sort_indices()
    return M


def maps_workload(cells=MAPS_CELLS, seed: int = SEED_MAPS, amp: float = MAPS_AMP):
    """Meshes (coarsest first) and the maps M(f_l): mesh l+1 -> mesh l of the non-nested
    workload: independently jittered grids of the given cell counts."""
    meshes = [jittered_grid(n, seed + 17 * k, amp) for k, n in enumerate(cells)]
    maps = [grid_point_location(meshes[k][0], meshes[k][1], cells[k], meshes[k + 1][0])
            for k in range(len(cells) - 1)]
    return meshes, maps


# ---------------------------------------------------------------- porous run of Sec. 3.2
# The paper's porous-convection experiment: a 16,641-vertex rectangle (128 x 128 cells, each
# split in two), Gaussian initial temperature (covariance I/2 around the centre, scaled by 400:
# peak 400/pi ~ 127), walls at +100 (bottom) and -100 (top), alpha rho0 = 1/g, phi = 0.1,
# Ra = 1000, k_etaf = 1, Delta T = 200, integrated to t = 0.5 with relative tolerance 1e-9.
# The extent of the rectangle is not printed; it is taken as [-20, 20] x [-20, 0] (40 x 20,
# the pedagogical setup the paper follows), see the design notes.
E4 = dict(base_cells=4, nsub=5, x_range=(-20.0, 20.0), y_range=(-20.0, 0.0), T_amp=400.0,
          cov=0.5, T_bottom=100.0, T_top=-100.0, Ra=1000.0, phi=0.1, delta_T=200.0,
          t_end=0.5, rtol=1e-9, atol=1e-6, n_save=10)


def e4_coords(xyz_unit: np.ndarray) -> np.ndarray:
    """Unit-square coordinates mapped affinely onto the E4 rectangle."""
    (x0, x1), (y0, y1) = E4["x_range"], E4["y_range"]
    out = np.array(xyz_unit, dtype=np.float64, copy=True)
    out[:, 0] = x0 + (x1 - x0) * out[:, 0]
    out[:, 1] = y0 + (y1 - y0) * out[:, 1]
    return out


def e4_initial_temperature(xyz: np.ndarray) -> np.ndarray:
    """T_amp times the bivariate normal density with mean at the centre of the rectangle and
    covariance cov * I, with the bottom wall at T_bottom and the top wall at T_top."""
    (x0, x1), (y0, y1) = E4["x_range"], E4["y_range"]
    cx, cy = 0.5 * (x0 + x1), 0.5 * (y0 + y1)
    s = E4["cov"]
    r2 = (xyz[:, 0] - cx) ** 2 + (xyz[:, 1] - cy) ** 2
    T = E4["T_amp"] / (2.0 * math.pi * s) * np.exp(-r2 / (2.0 * s))
    T[xyz[:, 1] == xyz[:, 1].min()] = E4["T_bottom"]
    T[xyz[:, 1] == xyz[:, 1].max()] = E4["T_top"]
    return T


def e4_save_times() -> np.ndarray:
    """Equally spaced save times in (0, t_end] for the error over time."""
    return E4["t_end"] * np.arange(1, E4["n_save"] + 1) / E4["n_save"]
