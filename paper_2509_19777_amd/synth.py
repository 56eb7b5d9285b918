"""Seeded synthetic inputs for hPLMM runs: voxel solids, stiffness fields,
box partitions, loads and random test vectors.

This module only *describes problems*.  It holds none of the method's
arithmetic (no stiffness, no assembly, no preconditioner); both the oracle and
the HIP library consume what it returns, each with its own code.

Voxel arrays have shape ``(nz, ny, nx)`` in C order, so the flat index of voxel
``(i, j, k)`` is ``i + nx * (j + ny * k)``: x runs fastest.  Lattice nodes are
numbered the same way on the ``(nx+1, ny+1, nz+1)`` node lattice.

The paper's own images (disk packs, sandstone, bone; Table 1) are not
available, so the workloads are synthetic stand-ins with the shapes stated by
the configurations:

* ``config_pores``: a cube with random non-overlapping spherical pores,
  homogeneous E, box subdomains (the 16^3 parity case).
* ``config_grf``: a cube whose solid phase is the top fraction of a Gaussian
  random field, with a lognormal E field (the 64^3 headline case).

Every solid is reduced to the 6-connected components that touch the clamped
plane z = 0, so the fine system has no floating or hinged parts.
"""
from __future__ import annotations

from dataclasses import dataclass, field

import numpy as np
from scipy import ndimage


@dataclass
class Problem:
    """A voxel elasticity problem and its subdomain partition.

    solid:    uint8 (nz, ny, nx), 1 = solid voxel kept in the model.
    E:        float64 (nz, ny, nx), Young's modulus per voxel (ignored on void).
    nu:       Poisson ratio (uniform).
    labels:   int32 (nz, ny, nx), subdomain (grain-grid) id per voxel, -1 on void.
    n_grains: number of subdomain ids (some may own no solid).
    traction: traction vector applied on the top face z = nz of every solid
              voxel in the top layer; the plane z = 0 is clamped.
    n_mortar: mortar nodes per interface (n in the paper).
    beta:     Gaussian mortar spread parameter.
    w_zeta:   contact-grid half width (Chebyshev lattice distance).
    name:     workload name.
    """

    solid: np.ndarray
    E: np.ndarray
    nu: float
    labels: np.ndarray
    n_grains: int
    traction: tuple = (0.0, 0.0, -1.0)
    n_mortar: int = 2
    beta: float = 4.0
    w_zeta: int = 1
    name: str = ""
    meta: dict = field(default_factory=dict)

    @property
    def shape(self):
        return self.solid.shape

    @property
    def dims(self):
        """(nx, ny, nz)."""
        nz, ny, nx = self.solid.shape
        return nx, ny, nz


def keep_clamped_components(solid: np.ndarray) -> np.ndarray:
    """Keep the 6-connected solid components that touch the plane z = 0."""
    lab, nlab = ndimage.label(solid.astype(bool))
    if nlab == 0:
        return np.zeros_like(solid, dtype=np.uint8)
    touching = np.unique(lab[0][lab[0] > 0])
    keep = np.isin(lab, touching)
    return keep.astype(np.uint8)


def box_labels(shape, box: int) -> tuple[np.ndarray, int]:
    """Cartesian decomposition into cubes of ``box`` voxels per side."""
    nz, ny, nx = shape
    bx, by, bz = -(-nx // box), -(-ny // box), -(-nz // box)
    k, j, i = np.meshgrid(np.arange(nz), np.arange(ny), np.arange(nx), indexing="ij")
    lab = (i // box) + bx * ((j // box) + by * (k // box))
    return lab.astype(np.int32), bx * by * bz


def sphere_pores(n: int, porosity: float, rmin: float, rmax: float, seed: int,
                 max_tries: int = 200000) -> np.ndarray:
    """Solid mask of an n^3 cube with random non-overlapping spherical pores.

    Centres are uniform in [0, n)^3 and radii uniform in [rmin, rmax]; a
    sphere overlapping an accepted one is rejected.  Voxels whose centre lies
    inside a sphere are void.  Spheres are added until the void fraction of
    voxel centres reaches ``porosity`` (or the attempt budget runs out).
    Each accepted sphere only touches the voxels of its bounding box, and the
    void count is kept incrementally.
    """
    rng = np.random.default_rng(seed)
    void = np.zeros((n, n, n), dtype=bool)
    n_void, total = 0, n ** 3
    # accepted spheres bucketed on a grid of cell 2 rmax: two spheres can
    # overlap only if their buckets are neighbours (the test itself is exact)
    cell = 2.0 * rmax
    nb = max(1, int(np.ceil(n / cell)))
    buckets = {}
    tries = 0
    while n_void < porosity * total and tries < max_tries:
        tries += 1
        p = rng.uniform(0.0, n, size=3)
        r = rng.uniform(rmin, rmax)
        b = tuple(min(nb - 1, int(p[d] // cell)) for d in range(3))
        hit = False
        for dz in (-1, 0, 1):
            for dy in (-1, 0, 1):
                for dx in (-1, 0, 1):
                    for q, s in buckets.get((b[0] + dx, b[1] + dy, b[2] + dz), ()):
                        if (p[0] - q[0]) ** 2 + (p[1] - q[1]) ** 2 + (p[2] - q[2]) ** 2 < (r + s) ** 2:
                            hit = True
                            break
                    if hit:
                        break
                if hit:
                    break
            if hit:
                break
        if hit:
            continue
        buckets.setdefault(b, []).append((p, r))
        lo = np.maximum(np.floor(p - r - 0.5).astype(int), 0)
        hi = np.minimum(np.ceil(p + r + 0.5).astype(int), n)
        cz = np.arange(lo[2], hi[2]) + 0.5
        cy = np.arange(lo[1], hi[1]) + 0.5
        cx = np.arange(lo[0], hi[0]) + 0.5
        inside = ((cx[None, None, :] - p[0]) ** 2 + (cy[None, :, None] - p[1]) ** 2
                  + (cz[:, None, None] - p[2]) ** 2) < r * r
        sub = void[lo[2]:hi[2], lo[1]:hi[1], lo[0]:hi[0]]
        n_void += int(np.count_nonzero(inside & ~sub))
        sub |= inside
    return (~void).astype(np.uint8)


def gaussian_field(n: int, ell: float, seed: int) -> np.ndarray:
    """Standardised periodic Gaussian random field on an n^3 voxel grid.

    White noise is convolved (by FFT, periodically) with a Gaussian kernel of
    standard deviation ell/2, which gives the covariance exp(-r^2/ell^2).
    """
    rng = np.random.default_rng(seed)
    w = rng.standard_normal((n, n, n))
    k = np.fft.fftfreq(n)
    KZ, KY, KX = np.meshgrid(k, k, k, indexing="ij")
    s = ell / 2.0
    filt = np.exp(-2.0 * (np.pi * s) ** 2 * (KX ** 2 + KY ** 2 + KZ ** 2))
    g = np.real(np.fft.ifftn(np.fft.fftn(w) * filt))
    g -= g.mean()
    g /= g.std()
    return g


def top_fraction(field_: np.ndarray, frac: float) -> np.ndarray:
    """Mask of the round(frac * size) largest values (ties to the lower index)."""
    flat = field_.ravel()
    m = int(round(frac * flat.size))
    order = np.argsort(-flat, kind="stable")
    mask = np.zeros(flat.size, dtype=np.uint8)
    mask[order[:m]] = 1
    return mask.reshape(field_.shape)


def _finish(solid, E, nu, box, name, **kw) -> Problem:
    solid = keep_clamped_components(solid)
    lab, ng = box_labels(solid.shape, box)
    lab = np.where(solid > 0, lab, -1).astype(np.int32)
    E = np.where(solid > 0, E, 0.0).astype(np.float64)
    return Problem(solid=solid, E=E, nu=nu, labels=lab, n_grains=ng, name=name, **kw)


def config_pores(n: int = 16, box: int = 4, seed: int = 1, porosity: float = 0.3,
                 n_mortar: int = 2, w_zeta: int = 1, traction=(0.0, 0.0, -1.0)) -> Problem:
    """Cube with spherical pores (radius 1-3), E = 1, nu = 0.3, box subdomains."""
    solid = sphere_pores(n, porosity, 1.0, 3.0, seed)
    E = np.ones(solid.shape)
    return _finish(solid, E, 0.3, box, f"pores{n}_box{box}_s{seed}", n_mortar=n_mortar,
                   w_zeta=w_zeta, traction=tuple(traction))


def config_grf(n: int = 64, box: int = 8, seed: int = 2, solid_frac: float = 0.6,
               ell: float = 6.0, sigma_lnE: float = 1.0, n_mortar: int = 2,
               w_zeta: int = 1, traction=(0.0, 0.0, -1.0)) -> Problem:
    """Cube whose solid is the top ``solid_frac`` of a Gaussian random field
    (correlation length ``ell``), ln E = sigma_lnE * (independent field)."""
    solid = top_fraction(gaussian_field(n, ell, seed), solid_frac)
    E = np.exp(sigma_lnE * gaussian_field(n, ell, seed + 1))
    return _finish(solid, E, 0.3, box, f"grf{n}_box{box}_s{seed}", n_mortar=n_mortar,
                   w_zeta=w_zeta, traction=tuple(traction))


def config_pores_lognormal(n: int = 64, box: int = 8, seed: int = 11, porosity: float = 0.3,
                           ell: float = 6.0, sigma_lnE: float = 1.0, n_mortar: int = 4,
                           w_zeta: int = 1, traction=(0.0, 0.0, -1.0)) -> Problem:
    """Spherical pores as in config_pores (radius 1-3) with a lognormal modulus
    ln E = sigma_lnE * (Gaussian random field of correlation length ``ell``):
    the subdomains the learned basis surrogate is trained and evaluated on."""
    solid = sphere_pores(n, porosity, 1.0, 3.0, seed)
    E = np.exp(sigma_lnE * gaussian_field(n, ell, seed + 1))
    return _finish(solid, E, 0.3, box, f"poresE{n}_box{box}_s{seed}", n_mortar=n_mortar,
                   w_zeta=w_zeta, traction=tuple(traction))


def voronoi_labels(shape, n_cells: int, seed: int) -> np.ndarray:
    """Irregular partition: every voxel takes the id of the nearest of n_cells
    seed points drawn uniformly in the cube (ties to the lower id)."""
    from scipy.spatial import cKDTree
    nz, ny, nx = shape
    rng = np.random.default_rng(seed)
    pts = rng.uniform(0.0, 1.0, size=(n_cells, 3)) * np.array([nx, ny, nz], dtype=float)
    k, j, i = np.meshgrid(np.arange(nz), np.arange(ny), np.arange(nx), indexing="ij")
    cen = np.stack([i.ravel() + 0.5, j.ravel() + 0.5, k.ravel() + 0.5], axis=1)
    _, idx = cKDTree(pts).query(cen, k=1)
    return idx.reshape(shape).astype(np.int32)


def disc_fractures(shape, n_fractures: int, seed: int, rmin: float, rmax: float) -> np.ndarray:
    """Mask of n_fractures planar discs one voxel thick: voxel centres within
    half a voxel of a random plane through a random centre and within a random
    radius of that centre."""
    nz, ny, nx = shape
    rng = np.random.default_rng(seed)
    k, j, i = np.meshgrid(np.arange(nz), np.arange(ny), np.arange(nx), indexing="ij")
    X = np.stack([i + 0.5, j + 0.5, k + 0.5], axis=-1)
    out = np.zeros(shape, dtype=bool)
    for _ in range(n_fractures):
        c = rng.uniform(0.0, 1.0, size=3) * np.array([nx, ny, nz], dtype=float)
        nrm = rng.standard_normal(3)
        nrm /= np.linalg.norm(nrm)
        r = rng.uniform(rmin, rmax)
        d = X - c
        h = d @ nrm
        rad = np.linalg.norm(d - h[..., None] * nrm, axis=-1)
        out |= (np.abs(h) < 0.5) & (rad < r)
    return out


def config_uneven(n: int = 128, seed: int = 31, porosity: float = 0.45, n_fractures: int = 5,
                  dofs_per_cell: float = 1000.0, n_mortar: int = 2, w_zeta: int = 1,
                  traction=(0.0, 0.0, -1.0), max_tries: int = 400000) -> Problem:
    """Uneven batching workload: spherical pores (radius 1-3, up to the given
    porosity or the attempt budget), n_fractures planar disc fractures as
    zero-stiffness (void) one-voxel layers, a two-phase modulus E in {1, 10}
    (thresholded Gaussian random field, correlation length 6), and an
    irregular Voronoi partition sized for about dofs_per_cell dofs per cell."""
    solid = sphere_pores(n, porosity, 1.0, 3.0, seed, max_tries=max_tries)
    solid[disc_fractures(solid.shape, n_fractures, seed + 1, n / 6.0, n / 3.0)] = 0
    solid = keep_clamped_components(solid)
    E = np.where(gaussian_field(n, 6.0, seed + 2) > 0.0, 10.0, 1.0)
    n_cells = max(2, int(round(3.3 * int(solid.sum()) / dofs_per_cell)))
    lab = voronoi_labels(solid.shape, n_cells, seed + 3)
    lab = np.where(solid > 0, lab, -1).astype(np.int32)
    E = np.where(solid > 0, E, 0.0).astype(np.float64)
    return Problem(solid=solid, E=E, nu=0.3, labels=lab, n_grains=n_cells, name=f"uneven{n}_s{seed}",
                   n_mortar=n_mortar, w_zeta=w_zeta, traction=tuple(traction))


def config_block(nx: int, ny: int, nz: int, box: int, E: float = 1.0, nu: float = 0.3,
                 holes=(), n_mortar: int = 2, w_zeta: int = 1,
                 traction=(0.0, 0.0, -1.0)) -> Problem:
    """A full (or hand-holed) nx x ny x nz block; ``holes`` lists (i, j, k) voids."""
    solid = np.ones((nz, ny, nx), dtype=np.uint8)
    for (i, j, k) in holes:
        solid[k, j, i] = 0
    Ef = np.full(solid.shape, float(E))
    return _finish(solid, Ef, nu, box, f"block{nx}x{ny}x{nz}_box{box}", n_mortar=n_mortar,
                   w_zeta=w_zeta, traction=tuple(traction))


def crop(problem: Problem, n: int, box: int = None) -> Problem:
    """The lower-corner n^3 sub-cube of a problem's fields (same plane z = 0
    clamped), re-filtered to components touching z = 0 and re-partitioned into
    boxes of the same size."""
    box = box or int(round(problem.solid.shape[0] / max(1, round(problem.n_grains ** (1 / 3)))))
    solid = problem.solid[:n, :n, :n].copy()
    E = problem.E[:n, :n, :n].copy()
    return _finish(solid, E, problem.nu, box, f"{problem.name}_crop{n}", n_mortar=problem.n_mortar,
                   w_zeta=problem.w_zeta, traction=tuple(problem.traction))


def random_vector(n: int, seed: int) -> np.ndarray:
    """Standard-normal float64 test vector."""
    return np.random.default_rng(seed).standard_normal(n)
