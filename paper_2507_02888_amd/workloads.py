"""Seeded synthetic workloads for the batched Ewald path.

This module defines the five benchmark systems (cells, particle counts, charges,
cutoffs, batch sizes) and draws every random input from a seeded generator:
walker positions, single-electron proposals, Metropolis accept flags, the walker
sizes of the uneven batch and the Jastrow coefficients. It contains none of the
Ewald arithmetic (no G vectors, no weights, no pair sums, no images): it is shared
by the oracle and by the HIP path, and both consume exactly the same arrays.

Units are Hartree atomic units (bohr, Ha), as in the paper's Sec. 1.

Workload readings (the paper measures VMC runs of homogeneous electron gases,
Sec. 5.2, and an hBN monolayer; those configurations come from a trial wave
function that is not available, so uniform-random positions stand in for them):

* cell volume from the density parameter r_s: Omega = (4 pi / 3) r_s^3 N_e in 3D,
  A = pi r_s^2 N_e in 2D; L = Omega^(1/3) (A^(1/2) in 2D);
* alpha = 5/L, real-space cutoff r_c = L/2, |G| <= m (2 pi / L) with m = 8
  (m = 12 for the N = 1024 system);
* positions s ~ U[0,1)^d in fractional coordinates, r = s A;
* move m of a walker moves electron k = m mod N_e to r' = r_k + sigma xi,
  xi ~ N(0, I_d), sigma = 0.3 bohr, Cartesian and unwrapped;
* accept iff u < p with u ~ U[0,1), independent of the energy change, so every
  implementation follows the same trajectory (p = 1 for the 54-electron system);
* streams of numpy.random.default_rng([2507, 2888, cfg, stream]): 0 positions,
  1 proposals, 2 accept uniforms, 3 walker sizes, 4 Jastrow coefficients.
"""
from __future__ import annotations

import dataclasses
import math
from typing import List, Optional

import numpy as np

SIGMA = 0.3
SEED = (2507, 2888)


def rng(cfg_id: int, stream: int) -> np.random.Generator:
    return np.random.default_rng([SEED[0], SEED[1], int(cfg_id), int(stream)])


# --------------------------------------------------------------------------
# cells (rows are lattice vectors; 2D cells use the upper-left 2x2 block)
# --------------------------------------------------------------------------

def sc_cell(volume: float) -> np.ndarray:
    c = volume ** (1.0 / 3.0)
    return c * np.eye(3)


def fcc_cell(volume: float) -> np.ndarray:
    c = (4.0 * volume) ** (1.0 / 3.0)  # conventional cube edge; primitive volume c^3/4
    return 0.5 * c * np.array([[0.0, 1.0, 1.0], [1.0, 0.0, 1.0], [1.0, 1.0, 0.0]])


def bcc_cell(volume: float) -> np.ndarray:
    c = (2.0 * volume) ** (1.0 / 3.0)  # primitive volume c^3/2
    return 0.5 * c * np.array([[-1.0, 1.0, 1.0], [1.0, -1.0, 1.0], [1.0, 1.0, -1.0]])


def hex_cell(area: float) -> np.ndarray:
    a = math.sqrt(area / (math.sqrt(3.0) / 2.0))
    m = np.zeros((3, 3))
    m[0, 0] = a
    m[1, 0] = 0.5 * a
    m[1, 1] = 0.5 * math.sqrt(3.0) * a
    m[2, 2] = 1.0  # unused third row for a 2D cell
    return m


def inscribed_radius(shape: str, measure: float) -> float:
    """Half the shortest nonzero lattice vector of the cells above (the radius
    of the sphere inscribed in the Wigner-Seitz cell), in closed form from
    the cell constructors: sc c, bcc c sqrt(3)/2, fcc c/sqrt(2), hex a."""
    if shape == "sc":
        return 0.5 * measure ** (1.0 / 3.0)
    if shape == "bcc":
        return 0.5 * (2.0 * measure) ** (1.0 / 3.0) * math.sqrt(3.0) / 2.0
    if shape == "fcc":
        return 0.5 * (4.0 * measure) ** (1.0 / 3.0) / math.sqrt(2.0)
    if shape == "hex":
        return 0.5 * math.sqrt(measure / (math.sqrt(3.0) / 2.0))
    raise ValueError(shape)


@dataclasses.dataclass
class System:
    """One periodic cell with its mobile electrons and fixed ions."""
    name: str
    dim: int
    lattice: np.ndarray          # [3][3], rows a_i (bohr)
    n_mobile: int
    mobile_q: np.ndarray         # [n_mobile]
    fixed_pos: np.ndarray        # [n_fixed][dim] Cartesian (bohr)
    fixed_q: np.ndarray          # [n_fixed]
    alpha: float
    r_cut: float
    g_cut: float
    # optional Jastrow two-body polynomial term u (Eq. (8)): coefficients
    # [2][N_u + 1] (channel 0: equal spin labels, 1: unequal), exponent C,
    # cutoff L_u, and a spin label (0/1) per mobile particle
    u_alpha: Optional[np.ndarray] = None
    u_C: int = 3
    u_cut: float = 0.0
    mobile_spin: Optional[np.ndarray] = None
    # optional layered 2D system (Eq. (5) with z != 0): heights of the planes
    # and the plane of each mobile particle (ascending) and fixed ion
    layer_z: Optional[np.ndarray] = None
    mobile_layer: Optional[np.ndarray] = None
    fixed_layer: Optional[np.ndarray] = None

    @property
    def n_fixed(self) -> int:
        return int(self.fixed_q.shape[0])

    @property
    def measure(self) -> float:
        """Cell volume (3D) or area (2D)."""
        return abs(float(np.linalg.det(self.lattice[: self.dim, : self.dim])))

    @property
    def length(self) -> float:
        return self.measure ** (1.0 / self.dim)


def _heg(name: str, dim: int, lattice: np.ndarray, n: int, gmul: float) -> System:
    a = lattice[:dim, :dim]
    L = abs(np.linalg.det(a)) ** (1.0 / dim)
    return System(name=name, dim=dim, lattice=lattice, n_mobile=n,
                  mobile_q=-np.ones(n), fixed_pos=np.zeros((0, dim)),
                  fixed_q=np.zeros(0), alpha=5.0 / L, r_cut=0.5 * L,
                  g_cut=gmul * 2.0 * math.pi / L)


DIAMOND_A0 = 10.2625  # bohr; the silicon lattice constant (5.431 Angstrom)


def diamond_supercell(k: int) -> System:
    """k x k x k multiple of the primitive fcc cell, two +4 ions per primitive
    cell at fractional (0,0,0) and (1/4,1/4,1/4) of the cubic edge, four
    electrons per ion."""
    prim = 0.5 * DIAMOND_A0 * np.array([[0.0, 1.0, 1.0], [1.0, 0.0, 1.0], [1.0, 1.0, 0.0]])
    lat = k * prim
    basis = [np.zeros(3), 0.25 * DIAMOND_A0 * np.ones(3)]
    ions = []
    for i in range(k):
        for j in range(k):
            for l in range(k):
                t = i * prim[0] + j * prim[1] + l * prim[2]
                for b in basis:
                    ions.append(t + b)
    ions = np.array(ions)
    n_e = 4 * len(ions)
    L = abs(np.linalg.det(lat)) ** (1.0 / 3.0)
    return System(name=f"diamond{k}", dim=3, lattice=lat, n_mobile=n_e,
                  mobile_q=-np.ones(n_e), fixed_pos=ions,
                  fixed_q=4.0 * np.ones(len(ions)), alpha=5.0 / L, r_cut=0.5 * L,
                  g_cut=8.0 * 2.0 * math.pi / L)


@dataclasses.dataclass
class Config:
    cfg_id: int
    description: str
    systems: List[System]
    walkers: int
    moves: int
    accept_p: float
    refresh_every: int            # K for the FP32-mixed form
    jastrow: bool = False
    max_jastrow_shells: int = 1024


def config(cfg_id: int) -> Config:
    if cfg_id == 1:
        n = 54
        sys_ = _heg("sc54", 3, sc_cell(4.0 / 3.0 * math.pi * n), n, 8.0)
        return Config(1, "3D HEG, simple-cubic cell, N=54, rs=1", [sys_], 1, 54, 1.0, 64)
    if cfg_id == 2:
        n = 250
        sys_ = _heg("fcc250", 3, fcc_cell(4.0 / 3.0 * math.pi * 8.0 * n), n, 8.0)
        return Config(2, "3D HEG, fcc-shaped cell, N=250, rs=2", [sys_], 1024, 256, 0.5, 64)
    if cfg_id == 3:
        n = 300
        sys_ = _heg("hex300", 2, hex_cell(math.pi * 25.0 * n), n, 8.0)
        return Config(3, "2D HEG, hexagonal cell, N=300, rs=5", [sys_], 2048, 512, 0.5, 64)
    if cfg_id == 4:
        return Config(4, "diamond fcc supercells 2x2x2/3x3x3/4x4x4, +4 ions",
                      [diamond_supercell(2), diamond_supercell(3), diamond_supercell(4)],
                      4096, 256, 0.5, 64)
    if cfg_id == 5:
        n = 1024
        sys_ = _heg("bcc1024", 3, bcc_cell(4.0 / 3.0 * math.pi * n), n, 12.0)
        return Config(5, "3D HEG, bcc-shaped cell, N=1024, rs=1, Jastrow plane-wave term",
                      [sys_], 8192, 1024, 0.5, 64, jastrow=True)
    raise ValueError(f"unknown config {cfg_id}")


@dataclasses.dataclass
class Batch:
    """Seeded inputs of one workload (possibly a subset of its walkers/moves)."""
    cfg: Config
    walker_sys: np.ndarray       # [W] int32, index into cfg.systems
    n_mobile: np.ndarray         # [W] int32
    pos_offsets: np.ndarray      # [W+1] int64, first particle of each walker
    pos: np.ndarray              # [P][dim] float64 Cartesian (packed)
    k: np.ndarray                # [S][W] int32
    new_pos: np.ndarray          # [S][W][dim] float64 Cartesian, unwrapped
    accept: np.ndarray           # [S][W] uint8
    jastrow_a: Optional[np.ndarray]  # [max_jastrow_shells] float64 or None

    @property
    def walkers(self) -> int:
        return int(self.walker_sys.shape[0])

    @property
    def steps(self) -> int:
        return int(self.k.shape[0])

    def walker_pos(self, w: int) -> np.ndarray:
        return self.pos[self.pos_offsets[w]: self.pos_offsets[w + 1]]


def make_batch(cfg: Config, walkers: Optional[int] = None, moves: Optional[int] = None,
               walker_start: int = 0) -> Batch:
    """Draw the seeded inputs. `walkers`/`moves` select a prefix subset; the
    draws for the full workload are made first so that every subset is a
    slice of the same full trajectory."""
    W_full, S_full = cfg.walkers, cfg.moves
    W = W_full if walkers is None else int(walkers)
    S = S_full if moves is None else int(moves)
    if not (0 <= walker_start and walker_start + W <= W_full and 0 <= S <= S_full):
        raise ValueError("subset out of range")
    dim = cfg.systems[0].dim
    # walker -> system
    if len(cfg.systems) == 1:
        wsys_full = np.zeros(W_full, dtype=np.int32)
    else:
        wsys_full = rng(cfg.cfg_id, 3).integers(0, len(cfg.systems), size=W_full).astype(np.int32)
    wsel = slice(walker_start, walker_start + W)
    wsys = wsys_full[wsel]
    nmob_full = np.array([cfg.systems[s].n_mobile for s in wsys_full], dtype=np.int64)
    # positions: fractional uniform, one block of draws per walker in order
    g0 = rng(cfg.cfg_id, 0)
    frac_full = g0.random((int(nmob_full.sum()), dim))
    off_full = np.zeros(W_full + 1, dtype=np.int64)
    off_full[1:] = np.cumsum(nmob_full)
    frac = frac_full[off_full[walker_start]: off_full[walker_start + W]]
    nmob = nmob_full[wsel]
    offs = np.zeros(W + 1, dtype=np.int64)
    offs[1:] = np.cumsum(nmob)
    pos = np.empty_like(frac)
    for w in range(W):
        lat = cfg.systems[wsys[w]].lattice[:dim, :dim]
        pos[offs[w]:offs[w + 1]] = frac[offs[w]:offs[w + 1]] @ lat
    # proposals and accept flags for the full move sequence (sliced below)
    xi = rng(cfg.cfg_id, 1).standard_normal((S_full, W_full, dim))[:S, wsel]
    u = rng(cfg.cfg_id, 2).random((S_full, W_full))[:S, wsel]
    acc = (u < cfg.accept_p).astype(np.uint8)
    k = np.empty((S, W), dtype=np.int32)
    new_pos = np.empty((S, W, dim))
    cur = pos.copy()
    widx = np.arange(W)
    for m in range(S):
        km = (m % nmob).astype(np.int64)
        k[m] = km
        rows = offs[:-1] + km
        prop = cur[rows] + SIGMA * xi[m]
        new_pos[m] = prop
        a = acc[m].astype(bool)
        cur[rows[a]] = prop[a]
    del widx
    ja = None
    if cfg.jastrow:
        ja = rng(cfg.cfg_id, 4).uniform(-0.01, 0.01, size=cfg.max_jastrow_shells)
    return Batch(cfg=cfg, walker_sys=wsys.astype(np.int32), n_mobile=nmob.astype(np.int32),
                 pos_offsets=offs, pos=pos, k=k, new_pos=new_pos, accept=acc, jastrow_a=ja)


def random_positions(system: System, n: int, seed: int) -> np.ndarray:
    """Uniform random Cartesian positions in a cell (for tests)."""
    g = np.random.default_rng([SEED[0], SEED[1], 99, int(seed)])
    d = system.dim
    return g.random((n, d)) @ system.lattice[:d, :d]


U_TERMS = 9   # N_u + 1 (the paper: N_u typically 8..12)
U_C = 3       # the paper: C = 2 or 3
CELL_SHAPE = {1: "sc", 2: "fcc", 3: "hex", 5: "bcc"}


def cusp_slope(dim: int, parallel: bool) -> float:
    """Kato cusp of the electron-electron Jastrow term, u'(0): 1/(d+1) for
    parallel and 1/(d-1) for antiparallel spins (unit charges and masses)."""
    return 1.0 / (dim + 1) if parallel else 1.0 / (dim - 1)


def with_u_term(system: System, cfg_id: int) -> System:
    """A copy of an electron-gas system with a seeded Jastrow u term (Eq. (8)):
    cutoff L_u = the Wigner-Seitz inscribed radius (as in the paper's HEG
    runs), C = 3, N_u = 8; coefficients alpha_l = x_l / L_u^(l+C) with
    x_l ~ U(-0.5, 0.5) (stream 5), except alpha_1, which is fixed by the cusp
    u'(0) = C alpha_0 (-L_u)^(C-1) + alpha_1 (-L_u)^C = Gamma; the first half
    of the electrons carry spin label 0, the rest 1."""
    Lu = inscribed_radius(CELL_SHAPE[cfg_id], system.measure)
    x = rng(cfg_id, 5).uniform(-0.5, 0.5, size=(2, U_TERMS))
    a = x / Lu ** (np.arange(U_TERMS)[None, :] + U_C)
    for c, parallel in ((0, True), (1, False)):
        gam = cusp_slope(system.dim, parallel)
        a[c, 1] = (gam - U_C * a[c, 0] * (-Lu) ** (U_C - 1)) / (-Lu) ** U_C
    n = system.n_mobile
    spin = np.concatenate([np.zeros(n // 2, dtype=np.int32), np.ones(n - n // 2, dtype=np.int32)])
    return dataclasses.replace(system, u_alpha=a, u_C=U_C, u_cut=Lu, mobile_spin=spin)


# Blip orbitals (Sec. 2.4): the N = 1024 bcc electron-gas cell with N/2 = 512
# orbitals per spin on a 40^3 grid (0.41 bohr spacing, about eight points per
# Fermi wavelength at r_s = 1), coefficients U(-1, 1) from stream 6 (no
# trained orbitals are available), evaluated at the workload's seeded
# proposals (one proposed position per walker and move).
BLIP_GRID = (40, 40, 40)
BLIP_ORBITALS = 512


def blip_coefficients(grid=BLIP_GRID, n_orb: int = BLIP_ORBITALS, seed_cfg: int = 5) -> np.ndarray:
    """Seeded blip coefficients [n1][n2][n3][n_orb] (float64)."""
    return rng(seed_cfg, 6).uniform(-1.0, 1.0, size=tuple(grid) + (int(n_orb),))


def blip_points(walkers: int, moves: int) -> np.ndarray:
    """Cartesian evaluation points [moves * walkers][3]: the proposals of the
    N = 1024 workload's first walkers and moves."""
    b = make_batch(config(5), walkers=walkers, moves=moves)
    return np.ascontiguousarray(b.new_pos.reshape(-1, 3))


def bilayer(n_each: int = 150, d: float = 5.0, rs: float = 5.0) -> System:
    """Electron-hole bilayer (Eq. (5) with z != 0): the hexagonal cell of the
    2D workload (area pi r_s^2 N for N = 2 n_each), n_each electrons
    (charge -1) in the plane z = 0 and n_each holes (charge +1) in the plane
    z = d; alpha = 5/L, r_c = L/2, |G| <= 8 (2 pi / L) as for the 2D gas."""
    n = 2 * n_each
    s = _heg(f"bilayer{n}", 2, hex_cell(math.pi * rs * rs * n), n, 8.0)
    q = np.concatenate([-np.ones(n_each), np.ones(n_each)])
    layer = np.concatenate([np.zeros(n_each, dtype=np.int32), np.ones(n_each, dtype=np.int32)])
    return dataclasses.replace(s, mobile_q=q, layer_z=np.array([0.0, float(d)]), mobile_layer=layer,
                               fixed_layer=np.zeros(0, dtype=np.int32))


def bilayer_config() -> Config:
    """The bilayer as a workload: 2048 walkers x 512 moves, p = 0.5, K = 64
    (seeds of the 2D gas, cfg 3, so positions and proposals are its draws)."""
    return Config(3, "electron-hole bilayer, hexagonal cell, 150 + 150 particles, d = r_s = 5",
                  [bilayer()], 2048, 512, 0.5, 64)
