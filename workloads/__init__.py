"""Seeded synthetic band endpoints for the CFNEB workloads.

This module only builds lattices and draws seeded noise; it holds none of the
method's arithmetic, so the CPU oracle and the HIP library can both be fed from
it.  All lengths in Angstrom; cells are 3x3 with lattice vectors as rows.

The paper's own systems (Ti3O5 with a machine-learned potential, graphite to
cubic diamond with an unnamed carbon potential, Sec. IV) are not reproducible
here; these workloads stand in with the same shapes:

* ``fcc_vacancy_hop``: Lennard-Jones FCC crystal with one vacancy; the final
  state is the nearest neighbour of the vacancy hopped into it.
* ``diamond_vacancy_hop``: the same hop in a cubic-diamond carbon crystal.
* ``graphite_to_diamond``: an orthorhombic AB-graphite supercell and the same
  atoms re-stacked ABC and puckered into a cubic-diamond-like (111) stacking,
  the shape of the graphite-to-diamond band of Sec. IV.B.
"""
import math

import numpy as np

FCC_BASIS = np.array([[0.0, 0.0, 0.0], [0.0, 0.5, 0.5], [0.5, 0.0, 0.5], [0.5, 0.5, 0.0]])


def fcc_sites(nx, ny, nz, a):
    """Site index ((ix*ny + iy)*nz + iz)*4 + b."""
    sites = []
    for ix in range(nx):
        for iy in range(ny):
            for iz in range(nz):
                for b in FCC_BASIS:
                    sites.append((np.array([ix, iy, iz]) + b) * a)
    cell = np.diag([nx * a, ny * a, nz * a])
    return np.array(sites), cell


def fcc_vacancy_hop(nx=4, ny=4, nz=4, a=1.5496):
    """Vacancy at site 0; atom k sits on site k+1.  In the final state atom 0
    (site 1, a nearest neighbour of site 0 at a/sqrt(2)) sits on site 0."""
    sites, cell = fcc_sites(nx, ny, nz, a)
    pos_i = sites[1:].copy()
    pos_f = pos_i.copy()
    pos_f[0] = sites[0]
    return dict(pos_init=pos_i, cell_init=cell.copy(), pos_final=pos_f, cell_final=cell.copy(),
                n=len(pos_i), types=np.zeros(len(pos_i), np.int32))


def diamond_vacancy_hop(nx=2, ny=2, nz=2, a=3.566):
    """Cubic diamond (8 sites per cube, site = cube*8 + b), vacancy at site 0.
    The hopping atom sits on site 4, the nearest neighbour (a/4)(1,1,1) of site 0."""
    basis = np.concatenate([FCC_BASIS, FCC_BASIS + 0.25])
    sites = []
    for ix in range(nx):
        for iy in range(ny):
            for iz in range(nz):
                for b in basis:
                    sites.append((np.array([ix, iy, iz]) + b) * a)
    sites = np.array(sites)
    cell = np.diag([nx * a, ny * a, nz * a])
    pos_i = sites[1:].copy()
    pos_f = pos_i.copy()
    pos_f[3] = sites[0]  # atom 3 is on site 4
    return dict(pos_init=pos_i, cell_init=cell.copy(), pos_final=pos_f, cell_final=cell.copy(),
                n=len(pos_i), types=np.zeros(len(pos_i), np.int32))


def _honeycomb_layers(nx, ny, nlayers, d, pitch, shift_of_layer, pucker):
    """Orthorhombic honeycomb stack.  Rectangle sqrt(3) d x 3 d holds 4 atoms at
    (0,0), (0,d), (sqrt3 d/2, 1.5 d), (sqrt3 d/2, 2.5 d); layer l is shifted by
    shift_of_layer(l) * d along y and its atoms move by pucker[b] along z.
    Atom index ((l*nx + ix)*ny + iy)*4 + b, the same in every stacking."""
    s3 = math.sqrt(3.0)
    base = np.array([[0.0, 0.0], [0.0, d], [s3 * d / 2, 1.5 * d], [s3 * d / 2, 2.5 * d]])
    Lx, Ly = nx * s3 * d, ny * 3.0 * d
    pos = []
    for layer in range(nlayers):
        sy = shift_of_layer(layer) * d
        for ix in range(nx):
            for iy in range(ny):
                for b in range(4):
                    x = base[b, 0] + ix * s3 * d
                    y = (base[b, 1] + iy * 3.0 * d + sy) % Ly
                    z = layer * pitch + pucker[b]
                    pos.append([x, y, z])
    cell = np.diag([Lx, Ly, nlayers * pitch])
    return np.array(pos), cell


def graphite_to_diamond(nx, ny, ncz, seed, sigma=0.01, d_graphite=1.46, pitch_graphite=3.35,
                        a_diamond=3.566):
    """AB graphite (2 layers per orthorhombic cell, ncz cells along z) to the same
    atoms in ABC stacking with (111)-diamond geometry.  ncz*2 must be a multiple of
    3 so that the ABC stacking is periodic.  Both endpoints get independent seeded
    N(0, sigma) displacements per atom and component (initial first, then final)."""
    nlayers = 2 * ncz
    if nlayers % 3 != 0:
        raise ValueError("2*ncz must be a multiple of 3 for a periodic ABC stacking")
    pos_i, cell_i = _honeycomb_layers(nx, ny, nlayers, d_graphite, pitch_graphite,
                                      lambda l: l % 2, [0.0, 0.0, 0.0, 0.0])
    d_dia = a_diamond / math.sqrt(6.0)      # in-plane projection of the diamond bond
    pitch_dia = a_diamond / math.sqrt(3.0)  # (111) bilayer pitch
    dz = a_diamond * math.sqrt(3.0) / 24.0  # half of the bilayer puckering
    # the atoms on (0, d) and (sqrt3 d/2, 2.5 d) sit under an atom of the next layer
    pos_f, cell_f = _honeycomb_layers(nx, ny, nlayers, d_dia, pitch_dia, lambda l: l % 3,
                                      [-dz, +dz, -dz, +dz])
    rng = np.random.default_rng(seed)
    pos_i = pos_i + rng.normal(0.0, sigma, pos_i.shape)
    pos_f = pos_f + rng.normal(0.0, sigma, pos_f.shape)
    return dict(pos_init=pos_i, cell_init=cell_i, pos_final=pos_f, cell_final=cell_f,
                n=len(pos_i), types=np.zeros(len(pos_i), np.int32))


# ----------------------------------------------------------------- recipes
def lj_fcc_hop_255():
    """LJ FCC 4x4x4 conventional cells, a = 1.5496 sigma, one vacancy: 255 atoms."""
    return fcc_vacancy_hop(4, 4, 4, 1.5496)


def tersoff_graphite_4608(seed=1):
    """Graphite to diamond-like, 4,608 atoms (12 x 8 rectangles, 12 layers)."""
    return graphite_to_diamond(12, 8, 6, seed)


def tersoff_graphite_98304(seed=2):
    """Graphite to diamond-like, 98,304 atoms (32 x 32 rectangles, 24 layers)."""
    return graphite_to_diamond(32, 32, 12, seed)


def small_graphite(nx=3, ny=2, ncz=3, seed=7):
    """A few-hundred-atom graphite band for fast parity tests."""
    return graphite_to_diamond(nx, ny, ncz, seed)


def random_cell(n, seed, density=0.08, skew=0.15, min_sep=0.0):
    """Random positions in a random triclinic cell (tests of neighbour sets)."""
    rng = np.random.default_rng(seed)
    vol = n / density
    L = vol ** (1.0 / 3.0)
    h = np.diag([L, L, L]) * (1.0 + 0.2 * (rng.random(3) - 0.5))
    h[1, 0] = skew * L * (rng.random() - 0.5)
    h[2, 0] = skew * L * (rng.random() - 0.5)
    h[2, 1] = skew * L * (rng.random() - 0.5)
    s = rng.random((n, 3))
    if min_sep > 0.0:
        # random sequential addition: redraw an atom closer than min_sep to an earlier
        # one (nearest periodic image)
        hinv = np.linalg.inv(h)
        for i in range(1, n):
            for _ in range(10000):
                ds = s[:i] - s[i]
                ds -= np.round(ds)
                if np.min(np.linalg.norm(ds @ h, axis=1)) >= min_sep:
                    break
                s[i] = rng.random(3)
        del hinv
    # unwrapped positions: some atoms sit one or two cells away
    s += rng.integers(-2, 3, size=(n, 3)) * (rng.random((n, 3)) < 0.1)
    return s @ h, h


# ------------------------------------------------------------ batches and streams
def _near_cubic(n_cells_target, lo=2):
    """(nx, ny, nz) with nx <= ny <= nz, aspect at most 2, product closest to the target."""
    best = None
    k = max(lo, int(round(n_cells_target ** (1.0 / 3.0))))
    for nx in range(max(lo, k - 3), k + 4):
        for ny in range(nx, 2 * nx + 1):
            for nz in range(ny, 2 * nx + 1):
                err = abs(nx * ny * nz - n_cells_target)
                if best is None or err < best[0]:
                    best = (err, (nx, ny, nz))
    return best[1]


def lj_hop_near(n_target):
    """LJ FCC vacancy hop with 4 nx ny nz - 1 atoms closest to n_target (cells >= 4 wide)."""
    nx, ny, nz = _near_cubic((n_target + 1) / 4.0, lo=4)
    return fcc_vacancy_hop(nx, ny, nz, 1.5496)


def diamond_hop_near(n_target):
    """Tersoff diamond vacancy hop with 8 nx ny nz - 1 atoms closest to n_target."""
    nx, ny, nz = _near_cubic((n_target + 1) / 8.0, lo=2)
    return diamond_vacancy_hop(nx, ny, nz)


def band_mix(seed, count, n_lo, n_hi, m_lo, m_hi, size_classes=0):
    """Independent bands: atom counts log-uniform in [n_lo, n_hi], image counts uniform in
    [m_lo, m_hi], LJ vacancy hops (even index) and Tersoff diamond vacancy hops (odd).
    size_classes > 0 snaps each drawn count to the nearest (in log) of that many
    log-spaced class sizes in [n_lo, n_hi], so that endpoints come from a pool of at
    most size_classes structures per family."""
    rng = np.random.default_rng(seed)
    classes = (np.exp(np.linspace(np.log(n_lo), np.log(n_hi), size_classes)) if size_classes > 0
               else None)
    out = []
    for q in range(count):
        n_target = float(np.exp(rng.uniform(np.log(n_lo), np.log(n_hi))))
        if classes is not None:
            n_target = float(classes[np.argmin(np.abs(np.log(classes) - np.log(n_target)))])
        m = int(rng.integers(m_lo, m_hi + 1))
        kind = "lj" if q % 2 == 0 else "ts"
        w = lj_hop_near(n_target) if kind == "lj" else diamond_hop_near(n_target)
        out.append(dict(kind=kind, n_images=m, endpoints=w, n=w["n"]))
    return out


def interior_noise(seed, n_images, n_atoms, sigma=0.01):
    """Seeded N(0, sigma) displacements (Angstrom) of every atom of the n_images - 2
    interior images of a band, shape (n_images - 2, n_atoms, 3), minus their mean.  They break the
    mirror symmetry of a straight-line start, which on the Tersoff vacancy hop sits on
    a ridge of the energy surface."""
    rng = np.random.default_rng(seed)
    d = rng.normal(0.0, sigma, size=(n_images - 2, n_atoms, 3))
    # zero mean per image: no rigid translation, which costs no energy and which the
    # springs of a periodic band would otherwise spread along the band
    return d - d.mean(axis=1, keepdims=True)


def poisson_arrivals(seed, count, rate):
    """Arrival times (s) of a Poisson stream of `count` requests at `rate` per second."""
    rng = np.random.default_rng(seed)
    return np.cumsum(rng.exponential(1.0 / rate, size=count))
