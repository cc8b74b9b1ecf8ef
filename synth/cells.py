"""Synthetic cells, Bloch-summed Gaussian basis functions and occupied orbitals.

Conventions (shared by every consumer of these inputs):

* Orthorhombic cell with edges ``L`` (bohr): lattice vectors a_i = L_i e_i,
  reciprocal vectors b_i = (2 pi / L_i) e_i, volume Omega = L1 L2 L3.
* Real-space grid ``(n1, n2, n3)``: point g = (g1, g2, g3) sits at
  r_g = sum_i (g_i / n_i) a_i; flat index (g1 * n2 + g2) * n3 + g3 (C order).
* k-mesh ``(N1, N2, N3)``, Gamma-centred unless ``kshift`` is set:
  k_n = sum_i ((n_i + s_i) / N_i) b_i, flat index n in C order.
* Basis function mu of k-point n (crystalline GTO, Sec. 1, Eq. 3 without the
  1/sqrt(N_k) factor): phi_mu^k(r) = sum_{R in {-1,0,1}^3} e^{i k.R}
  chi_mu(r - A_mu - R) with normalised Cartesian primitives
  s: (2a/pi)^{3/4} e^{-a r^2},  p_x: (2a/pi)^{3/4} 2 sqrt(a) x e^{-a r^2}.
  On an orthorhombic cell the image sum and the Gaussian both factorise over
  the three axes, so every function on the grid is an outer product of three
  1-D factors.
* Occupied orbitals: C^k = R^k (R^k^H S^k R^k)^{-1/2} with R^k iid standard
  complex normal and S^k = dV Phi^H Phi the grid overlap; psi_i^k = Phi^k C^k.
  Each orbital is then unit-normalised over the cell on the grid.
* Seeds: ``numpy.random.default_rng([230405505, config, cell])``; draw order
  geometry -> exponents -> R^k for every k in flat order.
"""

from __future__ import annotations

from dataclasses import dataclass, field

import numpy as np

SEED_ROOT = 230405505

# Benzene-crystal-like cell used for the molecular-crystal workloads (Sec. 4.3):
# orthorhombic 14.0 x 17.8 x 12.9 bohr holding four C6H6 rings.
RING_CELL_L = (14.0, 17.8, 12.9)
RING_CC = 2.64  # C-C bond (bohr) = radius of the carbon hexagon
RING_CH = 2.05  # C-H bond (bohr)
RING_CENTRES_4 = ((0.0, 0.0, 0.0), (0.5, 0.5, 0.0), (0.0, 0.5, 0.5), (0.5, 0.0, 0.5))
RING_CENTRES_2 = ((0.0, 0.0, 0.0), (0.5, 0.5, 0.5))
MIN_DIST = 1.5  # bohr, rejection threshold for any interatomic distance


@dataclass(frozen=True)
class Shell:
    atom: int
    l: int  # 0 = s, 1 = p (three Cartesian functions x, y, z)
    alpha: float


@dataclass
class Cell:
    name: str
    L: np.ndarray  # (3,) edges, bohr
    grid: tuple
    kmesh: tuple
    atoms: np.ndarray  # (n_atoms, 3) Cartesian positions inside [0, L)
    shells: list
    n_occ: int
    n_isdf: int
    kshift: np.ndarray = field(default_factory=lambda: np.zeros(3))
    R: list | None = None  # per-k random coefficient draws (N x n_occ)
    seed: tuple = ()

    @property
    def N_k(self) -> int:
        return int(np.prod(self.kmesh))

    @property
    def N_g(self) -> int:
        return int(np.prod(self.grid))

    @property
    def omega(self) -> float:
        return float(np.prod(self.L))

    @property
    def dV(self) -> float:
        return self.omega / self.N_g

    @property
    def functions(self) -> list:
        """Basis functions as (atom, (lx, ly, lz), alpha), shell order."""
        out = []
        for sh in self.shells:
            if sh.l == 0:
                out.append((sh.atom, (0, 0, 0), sh.alpha))
            elif sh.l == 1:
                for ax in range(3):
                    ang = [0, 0, 0]
                    ang[ax] = 1
                    out.append((sh.atom, tuple(ang), sh.alpha))
            else:
                raise ValueError("only s and p shells")
        return out

    @property
    def n_ao(self) -> int:
        return len(self.functions)

    def kvec(self, n: int) -> np.ndarray:
        idx = np.unravel_index(n, self.kmesh)
        return np.array(
            [(idx[i] + self.kshift[i]) / self.kmesh[i] * 2 * np.pi / self.L[i] for i in range(3)]
        )

    def kmesh_index(self, n: int) -> tuple:
        return tuple(int(v) for v in np.unravel_index(n, self.kmesh))


def smooth_grid_size(x: float) -> int:
    """Smallest 2*3*5-smooth integer >= x."""
    n = max(1, int(np.ceil(x - 1e-9)))
    while True:
        m = n
        for p in (2, 3, 5):
            while m % p == 0:
                m //= p
        if m == 1:
            return n
        n += 1


def grid_coords(cell: Cell, axis: int) -> np.ndarray:
    return np.arange(cell.grid[axis]) * (cell.L[axis] / cell.grid[axis])


def point_coords(cell: Cell, flat_idx) -> np.ndarray:
    """Cartesian coordinates (len, 3) of flat grid indices."""
    idx = np.unravel_index(np.asarray(flat_idx, dtype=np.int64), cell.grid)
    return np.stack([idx[i] * (cell.L[i] / cell.grid[i]) for i in range(3)], axis=-1)


# --------------------------------------------------------------------------
# geometry
# --------------------------------------------------------------------------

def _min_image_ok(pos: np.ndarray, L: np.ndarray, dmin: float) -> bool:
    d = pos[:, None, :] - pos[None, :, :]
    d -= L * np.round(d / L)
    r = np.sqrt((d * d).sum(-1))
    np.fill_diagonal(r, np.inf)
    return bool(r.min() >= dmin)


def _haar_rotation(rng: np.random.Generator) -> np.ndarray:
    a = rng.standard_normal((3, 3))
    q, r = np.linalg.qr(a)
    q = q * np.sign(np.diag(r))
    if np.linalg.det(q) < 0:
        q[:, 0] = -q[:, 0]
    return q


def _ring_local() -> tuple:
    ang = np.arange(6) * (np.pi / 3)
    ring = np.stack([np.cos(ang), np.sin(ang), np.zeros(6)], axis=-1)
    return ring * RING_CC, ring * (RING_CC + RING_CH)


def _place_rings(rng, L, centres_frac):
    c_loc, h_loc = _ring_local()
    local = np.concatenate([c_loc, h_loc])
    for _ in range(10000):
        pos = []
        for c in centres_frac:
            rot = _haar_rotation(rng)
            pos.append(np.asarray(c) * L + local @ rot.T)
        pos = np.mod(np.concatenate(pos), L)
        if _min_image_ok(pos, L, MIN_DIST):
            return pos
    raise RuntimeError("ring placement failed")


def _place_random(rng, L, n_atoms):
    for _ in range(100000):
        pos = rng.uniform(0.0, 1.0, size=(n_atoms, 3)) * L
        if _min_image_ok(pos, L, MIN_DIST):
            return pos
    raise RuntimeError("random placement failed")


# --------------------------------------------------------------------------
# exponents
# --------------------------------------------------------------------------

def _shells_sp(rng, n_atoms, lo=0.3, hi=1.2, fixed=None):
    shells = []
    for a in range(n_atoms):
        if fixed is not None:
            ea, eb = fixed, fixed
        else:
            ea, eb = rng.uniform(lo, hi, size=2)
        shells.append(Shell(a, 0, float(ea)))
        shells.append(Shell(a, 1, float(eb)))
    return shells


def _shells_2s2p(rng, n_atoms, lo=0.15, hi=2.0, ratio=1.5):
    def pair():
        for _ in range(10000):
            e = np.exp(rng.uniform(np.log(lo), np.log(hi), size=2))
            if max(e) / min(e) >= ratio:
                return sorted(e, reverse=True)
        raise RuntimeError("exponent draw failed")

    shells = []
    for a in range(n_atoms):
        s1, s2 = pair()
        p1, p2 = pair()
        shells += [Shell(a, 0, float(s1)), Shell(a, 0, float(s2)),
                   Shell(a, 1, float(p1)), Shell(a, 1, float(p2))]
    return shells


def _draw_R(rng, n_k, n_ao, n_occ):
    out = []
    for _ in range(n_k):
        re = rng.standard_normal((n_ao, n_occ))
        im = rng.standard_normal((n_ao, n_occ))
        out.append((re + 1j * im) / np.sqrt(2.0))
    return out


# --------------------------------------------------------------------------
# cell factories
# --------------------------------------------------------------------------

def make_random_cell(L, n_atoms, grid, kmesh, n_occ, n_isdf, seed, name="random",
                     alpha=None, kshift=(0.0, 0.0, 0.0)) -> Cell:
    """Atoms at uniform random positions, each with an s and a p shell."""
    L = np.asarray(L, dtype=np.float64)
    rng = np.random.default_rng(list(seed))
    atoms = _place_random(rng, L, n_atoms)
    shells = _shells_sp(rng, n_atoms, fixed=alpha)
    cell = Cell(name, L, tuple(grid), tuple(kmesh), atoms, shells, n_occ, n_isdf,
                kshift=np.asarray(kshift, dtype=np.float64), seed=tuple(seed))
    cell.R = _draw_R(rng, cell.N_k, cell.n_ao, n_occ)
    return cell


def make_ring_cell(L, centres, grid, kmesh, n_occ, n_isdf, seed, name="rings",
                   basis="sp", kshift=(0.0, 0.0, 0.0)) -> Cell:
    """C6H6 rings with Haar-random orientations at the given fractional centres."""
    L = np.asarray(L, dtype=np.float64)
    rng = np.random.default_rng(list(seed))
    atoms = _place_rings(rng, L, centres)
    if basis == "sp":
        shells = _shells_sp(rng, len(atoms))
    elif basis == "2s2p":
        shells = _shells_2s2p(rng, len(atoms))
    else:
        raise ValueError(basis)
    cell = Cell(name, L, tuple(grid), tuple(kmesh), atoms, shells, n_occ, n_isdf,
                kshift=np.asarray(kshift, dtype=np.float64), seed=tuple(seed))
    cell.R = _draw_R(rng, cell.N_k, cell.n_ao, n_occ)
    return cell


def make_config(config: int, cell_index: int = 0) -> Cell:
    """The five workload shapes (1-based numbering).

    1: Gamma only, cubic 8 bohr, 4 random atoms (s + p, exponent 0.8), 24^3 grid,
       n_occ 4, N_ISDF 64.
    2: 2x2x2 mesh, four-ring 48-atom cell, s + p per atom, 60x75x54 grid,
       n_occ 84, N_ISDF 420.
    3: as 2 on a 3x3x3 mesh.
    4: batched cells, see ``make_batch_cells``; ``cell_index`` picks one of 24.
    5: 4x4x4 mesh, four-ring cell with 2s + 2p per atom, 72x90x64 grid,
       n_occ 84, N_ISDF 420.
    """
    seed = (SEED_ROOT, config, cell_index)
    if config == 1:
        return make_random_cell((8.0, 8.0, 8.0), 4, (24, 24, 24), (1, 1, 1), 4, 64, seed,
                                name="config1-gamma", alpha=0.8)
    if config in (2, 3):
        km = (2, 2, 2) if config == 2 else (3, 3, 3)
        return make_ring_cell(RING_CELL_L, RING_CENTRES_4, (60, 75, 54), km, 84, 420, seed,
                              name=f"config{config}-rings-k{km[0]}")
    if config == 4:
        return make_batch_cells()[cell_index]
    if config == 5:
        return make_ring_cell(RING_CELL_L, RING_CENTRES_4, (72, 90, 64), (4, 4, 4), 84, 420,
                              seed, name="config5-rings-2s2p-k4", basis="2s2p")
    raise ValueError(config)


def make_config5_coarse() -> Cell:
    """Config 5's cell (4x4x4 mesh, four-ring cell with 2s + 2p per atom,
    n_occ 84, N_ISDF 420, the same seed) sampled on the coarser 36x45x32 grid:
    the 4x4x4 parity case whose FP64 oracle finishes in about an hour."""
    return make_ring_cell(RING_CELL_L, RING_CENTRES_4, (36, 45, 32), (4, 4, 4), 84, 420,
                          (SEED_ROOT, 5, 0), name="config5c-rings-2s2p-k4-coarse",
                          basis="2s2p")


def make_ring_series_cell(k: int) -> Cell:
    """The 48-atom four-ring cell of configs 2 and 3 (same geometry and basis,
    60x75x54 grid, n_occ 84, N_ISDF 420) on a k x k x k mesh: the N_k series."""
    return make_ring_cell(RING_CELL_L, RING_CENTRES_4, (60, 75, 54), (k, k, k), 84, 420,
                          (SEED_ROOT, 2, 0), name=f"rings-series-k{k}")


BATCH_ATOMS = (8, 16, 24, 48)
BATCH_KMESH = ((1, 1, 1), (2, 2, 2), (3, 3, 3))


def make_batch_cells() -> list:
    """24 cells: 2 x {8, 16, 24, 48 atoms} x {1^3, 2^3, 3^3} k-meshes.

    Cell volume scales with the atom count at the 48-atom density with the
    same aspect ratio; grids use the smallest 2*3*5-smooth size >= 4.5 points
    per bohr; 4 functions per atom; n_occ = round(0.44 N); N_ISDF = round(2.2 N).
    """
    cells = []
    idx = 0
    for rep in range(2):
        for na in BATCH_ATOMS:
            for km in BATCH_KMESH:
                seed = (SEED_ROOT, 4, idx)
                L = np.asarray(RING_CELL_L) * (na / 48.0) ** (1.0 / 3.0)
                grid = tuple(smooth_grid_size(4.5 * x) for x in L)
                n_ao = 4 * na
                n_occ = int(round(0.44 * n_ao))
                n_isdf = int(round(2.2 * n_ao))
                name = f"batch{idx}-a{na}-k{km[0]}"
                if na == 48:
                    c = make_ring_cell(L, RING_CENTRES_4, grid, km, n_occ, n_isdf, seed, name=name)
                elif na == 24:
                    c = make_ring_cell(L, RING_CENTRES_2, grid, km, n_occ, n_isdf, seed, name=name)
                else:
                    c = make_random_cell(L, na, grid, km, n_occ, n_isdf, seed, name=name)
                cells.append(c)
                idx += 1
    return cells


# --------------------------------------------------------------------------
# basis functions
# --------------------------------------------------------------------------

def _factors_1d(cell: Cell, kvec: np.ndarray, axis: int, x: np.ndarray) -> np.ndarray:
    """(n_ao, len(x)) complex: the per-axis factor of every basis function."""
    funcs = cell.functions
    out = np.zeros((len(funcs), len(x)), dtype=np.complex128)
    La = cell.L[axis]
    for mu, (atom, ang, alpha) in enumerate(funcs):
        A = cell.atoms[atom, axis]
        acc = np.zeros(len(x), dtype=np.complex128)
        for R in (-1, 0, 1):
            d = x - A - R * La
            val = np.exp(-alpha * d * d)
            if ang[axis] == 1:
                val = val * d
            acc += np.exp(1j * kvec[axis] * R * La) * val
        out[mu] = acc
    return out


def _norms(cell: Cell) -> np.ndarray:
    out = []
    for (_, ang, alpha) in cell.functions:
        c = (2 * alpha / np.pi) ** 0.75
        if sum(ang):
            c *= 2 * np.sqrt(alpha)
        out.append(c)
    return np.asarray(out)


def ao_on_grid(cell: Cell, n: int, dtype=np.complex128) -> np.ndarray:
    """phi_mu^{k_n}(r) on the full grid, shape (n_ao, N_g)."""
    k = cell.kvec(n)
    f = [_factors_1d(cell, k, a, grid_coords(cell, a)) for a in range(3)]
    nrm = _norms(cell)
    out = (nrm[:, None, None, None] * f[0][:, :, None, None]) * f[1][:, None, :, None]
    out = out * f[2][:, None, None, :]
    return out.reshape(cell.n_ao, cell.N_g).astype(dtype, copy=False)


def ao_at_points(cell: Cell, n: int, flat_idx) -> np.ndarray:
    """phi_mu^{k_n}(r_P) at flat grid indices, shape (n_ao, len(idx))."""
    k = cell.kvec(n)
    xyz = point_coords(cell, flat_idx)
    f = [_factors_1d(cell, k, a, xyz[:, a]) for a in range(3)]
    return _norms(cell)[:, None] * f[0] * f[1] * f[2]


def ao_overlap(cell: Cell, n: int) -> np.ndarray:
    """Grid overlap S^k = dV Phi^H Phi, computed axis by axis."""
    k = cell.kvec(n)
    nrm = _norms(cell)
    S = np.outer(nrm, nrm).astype(np.complex128)
    for a in range(3):
        f = _factors_1d(cell, k, a, grid_coords(cell, a))
        S *= (cell.L[a] / cell.grid[a]) * (f.conj() @ f.T)
    return S


def orbital_coeffs(cell: Cell, tr_symmetric: bool = False) -> list:
    """Loewdin-orthonormalised random coefficients C^k (n_ao x n_occ).

    With ``tr_symmetric`` the draws obey R^{-k} = conj(R^k) (real R at
    time-reversal-invariant k), so the orbitals obey psi^{-k} = conj(psi^k).
    """
    Rs = [r.copy() for r in cell.R]
    if tr_symmetric:
        if np.any(cell.kshift != 0):
            raise ValueError("time-reversal pairing assumes a Gamma-centred mesh")
        km = cell.kmesh
        for n in range(cell.N_k):
            idx = np.unravel_index(n, km)
            partner = int(np.ravel_multi_index(tuple((-i) % N for i, N in zip(idx, km)), km))
            if partner < n:
                Rs[n] = Rs[partner].conj()
            elif partner == n:
                Rs[n] = np.sqrt(2.0) * Rs[n].real + 0j
    out = []
    for n in range(cell.N_k):
        S = ao_overlap(cell, n)
        R = Rs[n]
        M = R.conj().T @ S @ R
        M = 0.5 * (M + M.conj().T)
        w, U = np.linalg.eigh(M)
        out.append(R @ (U * (1.0 / np.sqrt(w))) @ U.conj().T)
    return out


def orbitals_on_grid(cell: Cell, C: list, dtype=np.complex128) -> np.ndarray:
    """psi_i^{k_n}(r) = sum_mu C^k_{mu i} phi_mu^k(r), shape (N_k, n_occ, N_g)."""
    out = np.empty((cell.N_k, cell.n_occ, cell.N_g), dtype=dtype)
    for n in range(cell.N_k):
        phi = ao_on_grid(cell, n)
        out[n] = (C[n].T @ phi).astype(dtype, copy=False)
    return out
