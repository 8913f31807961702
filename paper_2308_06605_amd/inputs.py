"""Seeded synthetic inputs: hexahedral box meshes and initial states.

This module holds no arithmetic of the flux-reconstruction method itself. It only builds
the inputs that both the HIP library and the CPU oracle consume:

* mesh descriptions (corner vertex ids in VTK hexahedron order plus geometry nodes at the
  tensor Gauss-Lobatto-Legendre points of degree q, xi fastest),
* an optional smooth curving of the node coordinates,
* closed-form flow states (Taylor-Green vortex, isentropic vortex, uniform freestream)
  evaluated at caller-supplied physical coordinates.

The paper (section "FR Algorithm") states the method on unstructured hexahedra; its own
workloads (a turbine cascade and a cooled vane) are not available, so periodic boxes with
these closed-form states stand in for them.
"""
from __future__ import annotations

import dataclasses
import math

import numpy as np

# VTK hexahedron corner order: corner c sits at reference corner (bx, by, bz) in {0,1}^3.
VTK_CORNERS = np.array(
    [[0, 0, 0], [1, 0, 0], [1, 1, 0], [0, 1, 0], [0, 0, 1], [1, 0, 1], [1, 1, 1], [0, 1, 1]],
    dtype=np.int64,
)

GAMMA = 1.4
PRANDTL = 0.72


@dataclasses.dataclass
class Mesh:
    """A hexahedral mesh description.

    elem_vert  : int64 [E, 8], corner vertex ids in VTK order. Periodic images share one id.
    elem_nodes : float64 [E, (q+1)^3, 3], node coordinates at tensor GLL points of degree q,
                 reference index i + (q+1)*(j + (q+1)*k) (xi fastest).
    q          : geometry degree (>= 1).
    shape      : (nx, ny, nz) for box meshes, informational.
    lo, hi     : box corners, informational.
    """

    elem_vert: np.ndarray
    elem_nodes: np.ndarray
    q: int
    shape: tuple = ()
    lo: tuple = ()
    hi: tuple = ()

    @property
    def n_elem(self) -> int:
        return int(self.elem_vert.shape[0])


def gll_points(q: int) -> np.ndarray:
    """Gauss-Lobatto-Legendre points of degree q (q+1 points, ascending) via numpy."""
    if q < 1:
        raise ValueError("GLL needs q >= 1")
    inner = np.polynomial.legendre.Legendre.basis(q).deriv().roots()
    return np.concatenate([[-1.0], np.sort(np.real(inner)), [1.0]])


def curve_map(x: np.ndarray, amp: float, lo, hi, mode: str = "same") -> np.ndarray:
    """Smooth curving of node coordinates.

    mode "same" (the curved-mesh workload): every coordinate gets the same displacement
    amp*L*sin(2 pi xh) sin(2 pi yh) sin(2 pi zh), xh = (x - lo)/L box-normalised, L the box
    length along x. mode "mixed": the three coordinates get different displacements
    (wavenumber 2 along x, y, z respectively for dx, dy, dz), which makes the cross-product
    form of the metrics alias. Both vanish on the box faces, so periodic faces still match.
    """
    lo = np.asarray(lo, dtype=np.float64)
    hi = np.asarray(hi, dtype=np.float64)
    L = hi - lo
    xh = (x - lo) / L
    s = [np.sin(2 * np.pi * xh[..., c]) for c in range(3)]
    base = amp * L[0] * s[0] * s[1] * s[2]
    if mode == "same":
        return x + base[..., None]
    out = x.copy()
    for c in range(3):
        out[..., c] += base * np.cos(2 * np.pi * xh[..., c]) * 2.0
    return out


def box_mesh(n, lo=(0.0, 0.0, 0.0), hi=None, q: int = 1, periodic=(True, True, True),
             curve_amp: float = 0.0, curve_mode: str = "same") -> Mesh:
    """Uniform nx*ny*nz hexahedral box, optionally curved by `curve_map`.

    Element (ie, je, ke) has index ie + nx*(je + ny*ke). In a periodic direction the vertex
    lattice index wraps modulo n, so periodic images share a vertex id. At least 3 elements
    are needed across a periodic direction: with 2, the sorted corner ids of distinct faces
    coincide and the faces cannot be paired from vertex ids alone.
    """
    nx, ny, nz = (n, n, n) if np.isscalar(n) else tuple(int(v) for v in n)
    if hi is None:
        hi = (2 * np.pi, 2 * np.pi, 2 * np.pi)
    lo = np.asarray(lo, dtype=np.float64)
    hi = np.asarray(hi, dtype=np.float64)
    for nd, per in zip((nx, ny, nz), periodic):
        if per and nd < 3:
            raise ValueError("a periodic direction needs at least 3 elements")
    vx = nx if periodic[0] else nx + 1
    vy = ny if periodic[1] else ny + 1
    vz = nz if periodic[2] else nz + 1

    ie, je, ke = np.meshgrid(np.arange(nx), np.arange(ny), np.arange(nz), indexing="ij")
    ie = ie.transpose(2, 1, 0).reshape(-1)  # element index ie fastest
    je = je.transpose(2, 1, 0).reshape(-1)
    ke = ke.transpose(2, 1, 0).reshape(-1)
    E = nx * ny * nz

    cx = (ie[:, None] + VTK_CORNERS[None, :, 0]) % vx
    cy = (je[:, None] + VTK_CORNERS[None, :, 1]) % vy
    cz = (ke[:, None] + VTK_CORNERS[None, :, 2]) % vz
    elem_vert = (cx + vx * (cy + vy * cz)).astype(np.int64)

    r = (gll_points(q) + 1.0) / 2.0  # [0,1]
    h = (hi - lo) / np.array([nx, ny, nz], dtype=np.float64)
    # node (a, b, c) of element -> physical point, a fastest
    ra, rb, rc = np.meshgrid(r, r, r, indexing="ij")
    ra = ra.transpose(2, 1, 0).reshape(-1)
    rb = rb.transpose(2, 1, 0).reshape(-1)
    rc = rc.transpose(2, 1, 0).reshape(-1)
    nodes = np.empty((E, (q + 1) ** 3, 3), dtype=np.float64)
    nodes[:, :, 0] = lo[0] + h[0] * (ie[:, None] + ra[None, :])
    nodes[:, :, 1] = lo[1] + h[1] * (je[:, None] + rb[None, :])
    nodes[:, :, 2] = lo[2] + h[2] * (ke[:, None] + rc[None, :])
    if curve_amp != 0.0:
        nodes = curve_map(nodes, curve_amp, lo, hi, curve_mode)
    return Mesh(elem_vert=elem_vert, elem_nodes=np.ascontiguousarray(nodes), q=q,
                shape=(nx, ny, nz), lo=tuple(lo), hi=tuple(hi))


# ---------------------------------------------------------------------------------------------
# Closed-form states. xyz has shape [..., 3]; the result has shape [..., 5] holding the
# conserved variables (rho, rho u, rho v, rho w, E).
# ---------------------------------------------------------------------------------------------

def _conserved(rho, u, v, w, p, gamma=GAMMA):
    E = p / (gamma - 1.0) + 0.5 * rho * (u * u + v * v + w * w)
    return np.stack([rho, rho * u, rho * v, rho * w, E], axis=-1)


def tgv_state(xyz: np.ndarray, mach: float = 0.1, gamma: float = GAMMA) -> np.ndarray:
    """Taylor-Green vortex initial condition on [0, 2 pi)^3 with unit length, speed, density.

    u = sin x cos y cos z, v = -cos x sin y cos z, w = 0,
    p = p0 + (cos 2x + cos 2y)(cos 2z + 2)/16 with p0 = 1/(gamma Ma^2), rho = p/p0.
    """
    x, y, z = xyz[..., 0], xyz[..., 1], xyz[..., 2]
    p0 = 1.0 / (gamma * mach * mach)
    u = np.sin(x) * np.cos(y) * np.cos(z)
    v = -np.cos(x) * np.sin(y) * np.cos(z)
    w = np.zeros_like(u)
    p = p0 + (np.cos(2 * x) + np.cos(2 * y)) * (np.cos(2 * z) + 2.0) / 16.0
    rho = p / p0
    return _conserved(rho, u, v, w, p, gamma)


def vortex_state(xyz: np.ndarray, t: float = 0.0, beta: float = 5.0, center=(0.0, 0.0),
                 uinf=(1.0, 0.0), gamma: float = GAMMA, period=None) -> np.ndarray:
    """Isentropic vortex (an exact Euler solution advected with speed uinf).

    T = 1 - (gamma-1) beta^2/(8 gamma pi^2) exp(1 - r^2), rho = T^(1/(gamma-1)), p = rho T,
    du = -(beta/2pi)(y-yc) exp((1-r^2)/2), dv = (beta/2pi)(x-xc) exp((1-r^2)/2), w = 0.
    r is measured from the advected centre; with `period=(Lx, Ly)` the nearest periodic image
    of the centre is used.
    """
    x, y = xyz[..., 0], xyz[..., 1]
    xc = center[0] + uinf[0] * t
    yc = center[1] + uinf[1] * t
    dx = x - xc
    dy = y - yc
    if period is not None:
        dx = dx - period[0] * np.round(dx / period[0])
        dy = dy - period[1] * np.round(dy / period[1])
    r2 = dx * dx + dy * dy
    f = np.exp(0.5 * (1.0 - r2))
    u = uinf[0] - beta / (2 * np.pi) * dy * f
    v = uinf[1] + beta / (2 * np.pi) * dx * f
    w = np.zeros_like(u)
    T = 1.0 - (gamma - 1.0) * beta * beta / (8.0 * gamma * np.pi * np.pi) * f * f
    rho = T ** (1.0 / (gamma - 1.0))
    p = rho * T
    return _conserved(rho, u, v, w, p, gamma)


def freestream_state(xyz: np.ndarray, mach: float = 0.1, direction=(1.0, 0.5, 0.25),
                     gamma: float = GAMMA) -> np.ndarray:
    """Uniform flow: rho = 1, p = 1/(gamma Ma^2), |u| = Ma*c along `direction` (so |u| = 1)."""
    d = np.asarray(direction, dtype=np.float64)
    d = d / np.linalg.norm(d)
    p0 = 1.0 / (gamma * mach * mach)
    c0 = math.sqrt(gamma * p0)
    shape = xyz.shape[:-1]
    rho = np.ones(shape)
    vel = mach * c0 * d
    return _conserved(rho, rho * vel[0], rho * vel[1], rho * vel[2], p0 * rho, gamma)


def points_to_state_layout(Upts: np.ndarray) -> np.ndarray:
    """[E, Ns, 5] -> [E, 5, Ns] (the library layout: points innermost)."""
    return np.ascontiguousarray(np.transpose(Upts, (0, 2, 1)))


def state_from_coords(xyz_e3s: np.ndarray, fn, **kw) -> np.ndarray:
    """Evaluate a closed-form state at solution-point coordinates laid out [E, 3, Ns]."""
    pts = np.transpose(xyz_e3s, (0, 2, 1))
    return points_to_state_layout(fn(pts, **kw))


def random_smooth_perturbation(xyz_e3s: np.ndarray, seed: int, amp: float = 1e-3,
                               modes: int = 3, period=(2 * np.pi,) * 3) -> np.ndarray:
    """A seeded smooth random field [E, 5, Ns]: a few low Fourier modes per variable."""
    rng = np.random.default_rng(seed)
    pts = np.transpose(xyz_e3s, (0, 2, 1))
    out = np.zeros(pts.shape[:-1] + (5,))
    k0 = 2 * np.pi / np.asarray(period)
    for v in range(5):
        for _ in range(modes):
            k = rng.integers(1, 3, size=3) * k0
            ph = rng.uniform(0, 2 * np.pi)
            a = rng.normal()
            out[..., v] += a * np.sin(pts @ k + ph)
    return points_to_state_layout(amp * out)


def boundary_tags(mesh: Mesh, tag: int = 1) -> np.ndarray:
    """[E][6] int32: `tag` on every face whose sorted corner ids occur once in the mesh (a
    physical boundary), 0 elsewhere. Local face f lies at reference coordinate f//2 = -1 (even
    f) or +1 (odd f), with the VTK corner order."""
    E = mesh.elem_vert.shape[0]
    keys = {}
    for e in range(E):
        for f in range(6):
            d, s = f // 2, f % 2
            ids = tuple(sorted(int(mesh.elem_vert[e, c]) for c in range(8) if VTK_CORNERS[c][d] == s))
            keys.setdefault(ids, []).append((e, f))
    out = np.zeros((E, 6), dtype=np.int32)
    for lst in keys.values():
        if len(lst) == 1:
            out[lst[0]] = tag
    return out


def box_axis_points(mesh: Mesh, p: int):
    """The distinct solution-point coordinates along each axis of an uncurved box mesh: for
    axis d, n_d (p+1) values ordered (element index, point index)."""
    xs = np.polynomial.legendre.leggauss(p + 1)[0]
    out = []
    for d in range(3):
        h = (mesh.hi[d] - mesh.lo[d]) / mesh.shape[d]
        ie = np.arange(mesh.shape[d])
        out.append((mesh.lo[d] + h * (ie[:, None] + (xs[None, :] + 1.0) / 2.0)).ravel())
    return out


def grid_to_state_layout(G: np.ndarray, shape, p: int) -> np.ndarray:
    """A field on the tensor grid of box_axis_points, G[c][z][y][x], -> [E][c][Ns] with element
    ie + nx (je + ny ke) and point i + n (j + n k)."""
    nx, ny, nz = shape
    n = p + 1
    C = G.shape[0]
    T = G.reshape(C, nz, n, ny, n, nx, n)               # c, ke, k, je, j, ie, i
    T = np.transpose(T, (1, 3, 5, 0, 2, 4, 6))          # ke, je, ie, c, k, j, i
    return np.ascontiguousarray(T.reshape(nx * ny * nz, C, n ** 3))


def random_spectrum_state(mesh: Mesh, p: int, seed: int, k0: float = 3.0, kmax: int = 8,
                          energy: float = 0.125, mach: float = 0.1, gamma: float = GAMMA) -> np.ndarray:
    """A seeded divergence-free random-phase velocity field on the periodic box [0, 2 pi)^3 at
    uniform density 1 and pressure 1/(gamma Ma^2), as a state [E][5][Ns] on an uncurved box
    mesh at degree p.

    u(x) = sum_k Re(c_k exp(i k.x)) over integer wave vectors 0 < |k| <= kmax, with c_k a
    Gaussian complex vector projected normal to k (so div u = 0) and scaled so that the shell
    spectrum follows E(k) ~ k^4 exp(-2 (k/k0)^2); the field is then scaled to the mean kinetic
    energy `energy` (0.125, that of the Taylor-Green vortex) over the points with Gauss weights.
    Evaluated on the tensor grid of the solution points, one axis at a time.
    """
    rng = np.random.default_rng(seed)
    r = np.arange(-kmax, kmax + 1)
    KX, KY, KZ = np.meshgrid(r, r, r, indexing="ij")
    K = np.stack([KX, KY, KZ], axis=-1).astype(np.float64)
    kk = np.sqrt((K ** 2).sum(axis=-1))
    mask = (kk > 0) & (kk <= kmax)
    c = rng.normal(size=K.shape) + 1j * rng.normal(size=K.shape)
    kh = np.where(mask[..., None], K / np.where(kk > 0, kk, 1.0)[..., None], 0.0)
    c = c - kh * (c * kh).sum(axis=-1, keepdims=True)        # normal to k
    amp = np.where(mask, kk * np.exp(-((kk / k0) ** 2)), 0.0)  # |c|^2 ~ k^2 exp(-2 (k/k0)^2)
    c = c * amp[..., None]
    ax = box_axis_points(mesh, p)
    ex = [np.exp(1j * np.outer(r, a)) for a in ax]            # [2 kmax + 1][points on the axis]
    vel = []
    for comp in range(3):
        A = c[..., comp]                                        # [kx][ky][kz]
        T = np.einsum("abc,cz->abz", A, ex[2])
        T = np.einsum("abz,by->azy", T, ex[1])
        T = np.einsum("azy,ax->zyx", T, ex[0])
        vel.append(T.real)
    V = grid_to_state_layout(np.stack(vel), mesh.shape, p)      # [E][3][Ns]
    w = np.polynomial.legendre.leggauss(p + 1)[1]
    W = np.einsum("k,j,i->kji", w, w, w).ravel()
    ek = (0.5 * (V ** 2).sum(axis=1) * W).sum() / (W.sum() * V.shape[0])
    V *= np.sqrt(energy / ek)
    p0 = 1.0 / (gamma * mach * mach)
    U = np.empty((V.shape[0], 5, V.shape[2]))
    U[:, 0] = 1.0
    U[:, 1:4] = V
    U[:, 4] = p0 / (gamma - 1.0) + 0.5 * (V ** 2).sum(axis=1)
    return U


# ---------------------------------------------------------------------------------------------
# Invariance scrambler: random element relabelling plus a random proper rotation of each
# element's reference frame. The physical mesh and fields are unchanged; only their
# description is permuted, which exercises every relative face orientation.
# ---------------------------------------------------------------------------------------------

def cube_rotations():
    """The 24 proper rotations of the reference cube as signed permutation matrices."""
    import itertools

    mats = []
    for perm in itertools.permutations(range(3)):
        for signs in itertools.product((1, -1), repeat=3):
            M = np.zeros((3, 3), dtype=np.int64)
            for r in range(3):
                M[r, perm[r]] = signs[r]
            if round(np.linalg.det(M)) == 1:
                mats.append(M)
    return mats


def _rotated_index_map(npts: int, M: np.ndarray) -> np.ndarray:
    """For a symmetric tensor point set, new flat index -> old flat index under xi' = M xi."""
    idx = np.arange(npts)
    k, j, i = np.meshgrid(idx, idx, idx, indexing="ij")
    new = np.stack([i.ravel(), j.ravel(), k.ravel()], axis=0)  # flat index i fastest
    c_new = 2 * new - (npts - 1)
    c_old = M.T @ c_new
    old = (c_old + (npts - 1)) // 2
    return old[0] + npts * (old[1] + npts * old[2])


def scramble_mesh(mesh: Mesh, seed: int):
    """Return (new_mesh, info) with elements relabelled and each reference frame rotated.

    info = (order, rot) where new element e' is old element order[e'] seen through rotation
    matrix index rot[e'] of `cube_rotations()`.
    """
    rng = np.random.default_rng(seed)
    E = mesh.n_elem
    order = rng.permutation(E)
    mats = cube_rotations()
    rot = rng.integers(0, len(mats), size=E)
    q = mesh.q
    corner_lattice = {tuple(c): vi for vi, c in enumerate(VTK_CORNERS)}
    ev = np.empty_like(mesh.elem_vert)
    nodes = np.empty_like(mesh.elem_nodes)
    for e_new in range(E):
        e_old = order[e_new]
        M = mats[rot[e_new]]
        cmap = _rotated_index_map(2, M)
        for c_new in range(8):
            b = VTK_CORNERS[c_new]
            old_flat = cmap[b[0] + 2 * (b[1] + 2 * b[2])]
            ob = (old_flat % 2, (old_flat // 2) % 2, old_flat // 4)
            ev[e_new, c_new] = mesh.elem_vert[e_old, corner_lattice[ob]]
        nmap = _rotated_index_map(q + 1, M)
        nodes[e_new] = mesh.elem_nodes[e_old][nmap]
    new = Mesh(elem_vert=ev, elem_nodes=nodes, q=q, shape=mesh.shape, lo=mesh.lo, hi=mesh.hi)
    return new, (order, rot)


def scramble_field(X: np.ndarray, info, p: int) -> np.ndarray:
    """Apply a mesh scramble to a per-solution-point field laid out [E, C, (p+1)^3]."""
    order, rot = info
    mats = cube_rotations()
    out = np.empty_like(X)
    maps = {}
    for e_new in range(X.shape[0]):
        r = int(rot[e_new])
        if r not in maps:
            maps[r] = _rotated_index_map(p + 1, mats[r])
        out[e_new] = X[order[e_new]][:, maps[r]]
    return out
