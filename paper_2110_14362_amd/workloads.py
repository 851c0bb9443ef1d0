"""Seeded synthetic charge systems (inputs only; no part of the method).

These stand in for the paper's systems, which are not available here:
SPC/E bulk water (17,789 molecules in an 8.16 nm box, section 5.1) and a DPPC
membrane (section 5.2).  The generators reproduce their shapes: charge values,
rigid 3-site geometry, density, slab layering.  Every generator is a pure
function of its arguments and seed (numpy PCG64).

Each returns a dict with
    pos  (N, 3) float64 positions inside [0, box)
    q    (N,)   float64 charges (the system is neutral)
    mass (N,)   float64 masses
    box  (3,)   float64 side lengths
    name        short description
"""

import math

import numpy as np

# SPC/E-shaped rigid 3-site water (charges and geometry as in the configs)
Q_O = -0.8476
Q_H = 0.4238
R_OH = 1.0                                  # Angstrom
THETA_HOH = math.radians(109.47)
M_O = 15.9994
M_H = 1.008
WATER_PER_A3 = 0.033428                    # molecules per A^3 at 1 g/cm^3

# 1 g/cm^3 in molecules/A^3: 0.6022140857 / 18.01528 = 0.033428


def _rng(seed):
    return np.random.default_rng(np.random.PCG64(int(seed)))


def electrolyte(n=1000, box=(20.0, 20.0, 20.0), seed=1):
    """Primitive electrolyte: n/2 charges +1 then n/2 charges -1, uniform positions."""
    if n % 2:
        raise ValueError("electrolyte needs an even n")
    g = _rng(seed)
    box = np.asarray(box, dtype=np.float64)
    pos = g.random((n, 3)) * box
    q = np.where(np.arange(n) < n // 2, 1.0, -1.0)
    return dict(pos=pos, q=q, mass=np.ones(n), box=box, name="electrolyte N=%d" % n)


def _random_rotations(g, k):
    """k uniformly random rotation matrices (normalised 4-normal quaternions)."""
    qt = g.standard_normal((k, 4))
    qt /= np.linalg.norm(qt, axis=1, keepdims=True)
    w, x, y, z = qt.T
    R = np.empty((k, 3, 3))
    R[:, 0, 0] = 1 - 2 * (y * y + z * z)
    R[:, 0, 1] = 2 * (x * y - z * w)
    R[:, 0, 2] = 2 * (x * z + y * w)
    R[:, 1, 0] = 2 * (x * y + z * w)
    R[:, 1, 1] = 1 - 2 * (x * x + z * z)
    R[:, 1, 2] = 2 * (y * z - x * w)
    R[:, 2, 0] = 2 * (x * z - y * w)
    R[:, 2, 1] = 2 * (y * z + x * w)
    R[:, 2, 2] = 1 - 2 * (x * x + y * y)
    return R


def _water_molecules(g, oxygens, box):
    """Place randomly oriented rigid waters with oxygens at the given sites."""
    k = oxygens.shape[0]
    half = 0.5 * THETA_HOH
    ref = np.array([[0.0, 0.0, 0.0],
                    [R_OH * math.sin(half), 0.0, R_OH * math.cos(half)],
                    [-R_OH * math.sin(half), 0.0, R_OH * math.cos(half)]])
    R = _random_rotations(g, k)
    sites = oxygens[:, None, :] + np.einsum("kab,sb->ksa", R, ref)
    pos = np.mod(sites.reshape(-1, 3), box)
    q = np.tile([Q_O, Q_H, Q_H], k)
    mass = np.tile([M_O, M_H, M_H], k)
    return pos, q, mass


def water_box_side(n_mol):
    """Cubic side length holding n_mol waters at 1 g/cm^3."""
    return (n_mol / WATER_PER_A3) ** (1.0 / 3.0)


def water(n_mol=10000, box=None, seed=2, jitter=0.15):
    """Bulk-water-shaped charges: oxygens on a jittered simple-cubic lattice
    (n_mol sites drawn from the smallest cube lattice holding them),
    random orientations, cubic box at 1 g/cm^3 unless `box` is given."""
    g = _rng(seed)
    if box is None:
        L = water_box_side(n_mol)
        box = (L, L, L)
    box = np.asarray(box, dtype=np.float64)
    side = int(math.ceil(n_mol ** (1.0 / 3.0) - 1e-9))
    while side ** 3 < n_mol:
        side += 1
    idx = np.stack(np.meshgrid(np.arange(side), np.arange(side), np.arange(side),
                               indexing="ij"), -1).reshape(-1, 3)
    pick = g.permutation(idx.shape[0])[:n_mol]
    spacing = box / side
    ox = (idx[pick] + 0.5) * spacing + g.uniform(-jitter, jitter, (n_mol, 3))
    pos, q, mass = _water_molecules(g, ox, box)
    return dict(pos=pos, q=q, mass=mass, box=box, name="water %d molecules" % n_mol)


def membrane_slab(box=(80.0, 80.0, 100.0), n_head=1024, sheet_offset=20.0, dipole=1.0,
                  water_gap=25.0, seed=3, jitter=0.15):
    """Membrane-shaped slab: two headgroup sheets at z = zc -/+ sheet_offset, each
    n_head dipoles (-1 at the sheet, +1 `dipole` above it, lateral positions
    uniform); waters fill |z - zc| > water_gap at 1 g/cm^3.  zc = box_z/2."""
    g = _rng(seed)
    box = np.asarray(box, dtype=np.float64)
    zc = 0.5 * box[2]
    heads_pos, heads_q = [], []
    for zs in (zc - sheet_offset, zc + sheet_offset):
        xy = g.random((n_head, 2)) * box[:2]
        neg = np.column_stack([xy, np.full(n_head, zs)])
        pos_ = np.column_stack([xy, np.full(n_head, zs + dipole)])
        heads_pos += [neg, pos_]
        heads_q += [np.full(n_head, -1.0), np.full(n_head, 1.0)]
    n_water = int(round(WATER_PER_A3 * box[0] * box[1] * (box[2] - 2 * water_gap)))
    a = WATER_PER_A3 ** (-1.0 / 3.0)
    nxy = int(round(box[0] / a))
    nz = int(round(box[2] / a))
    idx = np.stack(np.meshgrid(np.arange(nxy), np.arange(nxy), np.arange(nz), indexing="ij"),
                   -1).reshape(-1, 3)
    spacing = np.array([box[0] / nxy, box[1] / nxy, box[2] / nz])
    centers = (idx + 0.5) * spacing
    ok = np.abs(centers[:, 2] - zc) > water_gap
    cand = centers[ok]
    if cand.shape[0] < n_water:
        raise ValueError("lattice too coarse for the water count")
    pick = g.permutation(cand.shape[0])[:n_water]
    ox = cand[pick] + g.uniform(-jitter, jitter, (n_water, 3))
    wpos, wq, wm = _water_molecules(g, ox, box)
    pos = np.vstack(heads_pos + [wpos])
    q = np.concatenate(heads_q + [wq])
    mass = np.concatenate([np.full(4 * n_head, 1.0), wm])
    pos = np.mod(pos, box)
    return dict(pos=pos, q=q, mass=mass, box=box,
                name="membrane slab %d head charges + %d waters" % (4 * n_head, n_water))


def nacl_crystal(cells=1, a=1.0):
    """Rocksalt crystal of cells^3 conventional cells; nearest-neighbour distance a."""
    L = 2.0 * a
    base_na = np.array([[0, 0, 0], [0, .5, .5], [.5, 0, .5], [.5, .5, 0]])
    base_cl = base_na + np.array([.5, 0, 0])
    pos, q = [], []
    for i in range(cells):
        for j in range(cells):
            for k in range(cells):
                off = np.array([i, j, k], dtype=np.float64)
                pos += [(base_na + off) * L, (np.mod(base_cl, 1.0) + off) * L]
                q += [np.ones(4), -np.ones(4)]
    pos = np.vstack(pos)
    box = np.full(3, cells * L)
    q = np.concatenate(q)
    return dict(pos=pos, q=q, mass=np.ones(len(q)), box=box, name="NaCl %d^3 cells" % cells)


def random_neutral(n, box, seed, qscale=1.0):
    """n random charges (n even): n/2 random magnitudes and their negatives."""
    g = _rng(seed)
    box = np.asarray(box, dtype=np.float64)
    half = g.uniform(0.2, 1.0, n // 2) * qscale
    q = np.concatenate([half, -half])
    if n % 2:
        q = np.concatenate([q, [0.0]])
    g.shuffle(q)
    pos = g.random((n, 3)) * box
    return dict(pos=pos, q=q, mass=np.ones(n), box=box, name="random neutral N=%d" % n)


# ---------------------------------------------------------------------------
# the workloads of the configurations (sizes and parameters)

CONFIGS = {
    # primitive electrolyte, reduced units, g = 0.3 (alpha = 0.09), r_c = 6, P = 100
    "electrolyte_1k": dict(kind="electrolyte", n=1000, L=20.0, g=0.3, rc=6.0, p=100,
                           coulomb=1.0, seed=2110143621),
    # bulk-water-shaped, 10,000 molecules at 1 g/cm^3 (L = 66.88 A), g = 0.3/A, P = 100
    "water_30k": dict(kind="water", n_mol=10000, g=0.3, rc=10.0, p=100,
                      coulomb=332.0637, seed=2110143622),
    # membrane-shaped slab 80 x 80 x 100 A, P = 200, semi-isotropic
    "slab_36k": dict(kind="slab", g=0.3, rc=10.0, p=200, coulomb=332.0637, seed=2110143623),
    # precision sweep at scale: 333,333 molecules (N = 999,999), L = 215.24 A
    "water_1m": dict(kind="water", n_mol=333333, g=0.3, rc=10.0, p=2000,
                     coulomb=332.0637, seed=2110143624),
}


def make(name, **over):
    """Build the system of a named configuration (see CONFIGS)."""
    c = dict(CONFIGS[name])
    c.update(over)
    if c["kind"] == "electrolyte":
        s = electrolyte(c["n"], (c["L"],) * 3, seed=c["seed"])
    elif c["kind"] == "water":
        s = water(c["n_mol"], seed=c["seed"])
    elif c["kind"] == "slab":
        s = membrane_slab(seed=c["seed"])
    else:
        raise KeyError(c["kind"])
    s.update(alpha=c["g"] ** 2, g=c["g"], rc=c["rc"], p=c["p"], coulomb=c["coulomb"],
             config=name)
    return s


# ---------------------------------------------------------------------------
# NPT parameters in real units (A, fs, kcal/mol, g/mol, e)

KB_KCAL = 0.0019872043              # kcal/mol/K
FTM_REAL = 4.184e-4                 # kcal/mol/A -> (g/mol) A / fs^2
ATM_KCAL_A3 = 101325.0 / 6.9477e9   # 1 atm in kcal/mol/A^3
KBAR_PER_KCAL_A3 = 69.477           # 1 kcal/mol/A^3 in kbar
COULOMB_REAL = 332.0637             # kcal A / (mol e^2)


def npt_real(box, T=300.0, p_atm=1.0, dt=1.0, tau_p=100.0, tau_cell=500.0, beta_kbar=4.5e-2,
             rc=10.0, box_mode="iso"):
    """Langevin NPT parameters for a real-unit system: particle friction
    1/tau_p, cell friction 1/tau_cell, barostat mass M = tau_cell^2 / (beta_T V0)
    (beta_T the isothermal compressibility in the integrator's pressure units),
    so that gamma_cell M = tau_cell / (beta_T V0)."""
    V0 = float(np.prod(box))
    beta = beta_kbar * KBAR_PER_KCAL_A3 / FTM_REAL          # (A fs^2 mol/g)
    M = tau_cell ** 2 / (beta * V0)
    d = dict(dt=dt, kT=KB_KCAL * T, p_ext=p_atm * ATM_KCAL_A3, gamma_p=1.0 / tau_p,
             gamma_cell=1.0 / tau_cell, mass_cell=M, mass_cell_z=0.0, ftm=FTM_REAL,
             box_mode=box_mode, rc=rc)
    if box_mode == "semiiso":
        A0 = box[0] * box[1]
        d["mass_cell"] = tau_cell ** 2 / (beta * V0) * box[2] ** 2
        d["mass_cell_z"] = tau_cell ** 2 / (beta * V0) * A0 ** 2
    return d


# ---------------------------------------------------------------------------
# served mixed-size stream

CHARGES_PER_A3 = 3.0 * WATER_PER_A3  # 0.100284 charges per A^3 (water at 1 g/cm^3)
ION_MASSES = (22.99, 35.45)          # cation, anion (g/mol)
ION_SIGMA, ION_EPS = 1.7, 1.0        # repulsive core 4 eps (sigma/r)^12 (A, kcal/mol)
EPS_WATER = 78.5                     # primitive model: the solvent as a dielectric continuum


def splitmix64(x):
    """SplitMix64 output for state x (sub-seed derivation)."""
    m = (1 << 64) - 1
    z = (x + 0x9E3779B97F4A7C15) & m
    z = ((z ^ (z >> 30)) * 0xBF58476D1CE4E5B9) & m
    z = ((z ^ (z >> 27)) * 0x94D049BB133111EB) & m
    return z ^ (z >> 31)


def ions(n, box, seed, jitter=0.15):
    """Primitive electrolyte with a repulsive core: n ions (n/2 at +1, n/2 at
    -1, in random order) on a jittered lattice filling the rectangular box
    (so no two start closer than the lattice spacing minus 2 jitter).  The
    caller sets the Coulomb constant (the primitive model divides it by the
    solvent's relative permittivity)."""
    g = _rng(seed)
    box = np.asarray(box, dtype=np.float64)
    # lattice with about n sites, spacing about equal on the three axes
    a = (np.prod(box) / n) ** (1.0 / 3.0)
    dims = np.maximum(1, np.ceil(box / a).astype(int))
    while np.prod(dims) < n:
        dims[np.argmax(box / dims)] += 1
    idx = np.stack(np.meshgrid(*[np.arange(d) for d in dims], indexing="ij"), -1).reshape(-1, 3)
    pick = g.permutation(idx.shape[0])[:n]
    spacing = box / dims
    pos = np.mod((idx[pick] + 0.5) * spacing + g.uniform(-jitter, jitter, (n, 3)), box)
    q = np.where(np.arange(n) < n // 2, 1.0, -1.0)
    g.shuffle(q)
    mass = np.where(q > 0, ION_MASSES[0], ION_MASSES[1])
    c12 = 4.0 * ION_EPS * ION_SIGMA ** 12
    lj = np.array([[[c12, 0.0]]])
    return dict(pos=pos, q=q, mass=mass, box=box, types=np.zeros(n, dtype=np.int32), lj=lj,
                name="ions N=%d" % n)


def serving_request(i, seed=2110143625, nmin=1000, nmax=200000, p=100, steps=20, g_ewald=0.3,
                    rc=10.0, kinds=("ions", "water")):
    """Request i of the served stream: N log-uniform in [nmin, nmax], kind
    drawn from `kinds` (ions or rigid 3-site water), cubic or 1:1:1.25 box
    (fair coin) at 0.100284 charges per A^3, P frequencies, `steps` NPT steps.
    Boxes shorter than 3.3 rc get a cutoff of a third of their shortest side
    less 10 % and a splitting parameter g = g_ewald rc / rc' that keeps
    erfc(g rc) (the real-space truncation error) unchanged."""
    sub = splitmix64((seed + i) & ((1 << 64) - 1))
    g = _rng(sub)
    n = int(round(math.exp(g.uniform(math.log(nmin), math.log(nmax)))))
    kind = kinds[int(g.integers(len(kinds)))]
    aspect = np.array([1.0, 1.0, 1.25]) if g.integers(2) else np.ones(3)
    if kind == "water":
        n_mol = max(n // 3, 1)
        n = 3 * n_mol
    else:
        n += n % 2
    L = (n / CHARGES_PER_A3 / np.prod(aspect)) ** (1.0 / 3.0)
    box = aspect * L
    if kind == "water":
        s = rigid_water(n_mol, box, seed=sub)
    else:
        s = ions(n, box, seed=sub)
    rc_i = min(rc, float(box.min()) / 3.3)
    g_i = g_ewald * rc / rc_i
    # the primitive electrolyte's ions interact through the solvent's dielectric
    coul = COULOMB_REAL if kind == "water" else COULOMB_REAL / EPS_WATER
    s.update(alpha=g_i ** 2, g=g_i, rc=rc_i, p=p, coulomb=coul, kind=kind, steps=steps,
             request=i, seed=sub)
    return s


def list_skin(box, rc, skin, margin=2.6):
    """The real-space neighbour-list skin a box allows: at most `skin`, with
    margin x (rc + skin) within the shortest side (the kernels need 2.5; the
    rest leaves room for the barostat to shrink the cell); 0 (no lists) when
    less than a tenth of an angstrom would remain."""
    s = min(float(skin), float(np.min(box)) / margin - rc)
    return s if s >= 0.1 else 0.0


# SPC/E oxygen-oxygen Lennard-Jones (sigma 3.166 A, epsilon 0.650 kJ/mol)
SPCE_SIGMA, SPCE_EPS = 3.166, 0.1553   # A, kcal/mol
D_OH = R_OH
D_HH = 2.0 * R_OH * math.sin(0.5 * THETA_HOH)


def water_lj(n_atoms, first=0, n_mol=None):
    """Types (O = 0, H = 1, anything before `first` = 2) and the LJ table
    lj[ti][tj] = (c12, c6) with only the O-O pair non-zero."""
    if n_mol is None:
        n_mol = (n_atoms - first) // 3
    types = np.full(n_atoms, 2, dtype=np.int32)
    types[first:first + 3 * n_mol] = np.tile([0, 1, 1], n_mol)
    lj = np.zeros((3, 3, 2))
    lj[0, 0] = (4.0 * SPCE_EPS * SPCE_SIGMA ** 12, 4.0 * SPCE_EPS * SPCE_SIGMA ** 6)
    return types, lj


def whole_molecules(pos, box, first, n_mol):
    """Positions with every rigid molecule's H atoms moved to the image
    nearest its O (the constraint solvers need whole molecules)."""
    pos = np.array(pos, dtype=np.float64)
    box = np.asarray(box, dtype=np.float64)
    o = pos[first:first + 3 * n_mol:3]
    for j in (1, 2):
        h = pos[first + j:first + 3 * n_mol:3]
        d = h - o
        pos[first + j:first + 3 * n_mol:3] = o + d - box * np.rint(d / box)
    return pos


def rigid_water(n_mol, box=None, seed=2):
    """water() with whole molecules (H atoms beside their O, not wrapped),
    SPC/E O-O Lennard-Jones types and the rigid-molecule description."""
    s = water(n_mol, box=box, seed=seed)
    s["pos"] = whole_molecules(s["pos"], s["box"], 0, n_mol)
    types, lj = water_lj(3 * n_mol)
    s.update(types=types, lj=lj, rigid=dict(first=0, count=n_mol, d_oh=D_OH, d_hh=D_HH))
    return s
