"""Seeded synthetic inputs shared by the oracle, the tests and the benchmark.

This module makes inputs only: geometries, model hyper-parameters and network
weights.  It holds none of the potential's arithmetic (no cutoff function, no
symmetry function, no network evaluation), so that the FP64 oracle and the HIP
path, which share no code, can both be fed from it.

Workloads (all synthetic; the paper's water-box benchmark of its Table S3 and
its ML/MM systems are stood in for by these generators):

* ``water_box``     liquid-water boxes at 1.0 g/cm^3: rigid-geometry TIP3P-like
                    molecules (O-H 0.9572 A, H-O-H 104.52 deg) with oxygens on a
                    cubic lattice, +-0.3 A uniform jitter and uniformly random
                    orientations (Shoemake quaternions).
* ``walk_molecule`` non-periodic H/C/N/O molecules grown by a self-avoiding
                    random walk (bond 1.0-1.5 A, no pair closer than 0.9 A).
* ``solute_in_water`` a walk solute embedded in fixed-charge MM water.
* ``model_config`` / ``model_weights``: the frozen hyper-parameters of the
                    ANI-style descriptor and the per-element networks, and
                    Xavier-normal weights drawn from a counter-based generator
                    (SplitMix64 + Box-Muller) that the C library re-implements
                    from the same published definition for its seed path.
"""
from __future__ import annotations

import math

import numpy as np

__all__ = [
    "model_config", "model_weights", "flat_weights", "splitmix64", "uniform01",
    "water_box", "walk_molecule", "walk_batch", "solute_in_water", "maxwell_boltzmann",
    "WATER_MASS", "KE_COULOMB", "KB_EV", "ACC_UNIT", "lj_params_solute", "lj_params_water",
]

# Units: Angstrom, eV, elementary charge, amu, fs.
KE_COULOMB = 14.3996454784      # eV * A / e^2
KB_EV = 8.617333262e-5          # eV / K
ACC_UNIT = 9.64853321233e-3     # (eV / (A * amu)) -> A / fs^2
WATER_MASS = {1: 1.008, 6: 12.011, 7: 14.007, 8: 16.00}

_OH = 0.9572
_HOH = math.radians(104.52)


# --------------------------------------------------------------------------
# Model hyper-parameters (frozen readings; every float is stored as the FP32
# value the GPU receives, so both sides see identical inputs).
# --------------------------------------------------------------------------
def model_config(kind: str = "water") -> dict:
    """Return the descriptor/network hyper-parameters of one model form.

    kind: "water"  -- species {H, O}, 128-dim descriptor, 128-160-128-96-1 MLP;
          "hcno"   -- species {H, C, N, O}, 384-dim descriptor, 384-256-192-160-1;
          "hcno_mm"-- as "hcno" plus one extra input (the MM electrostatic
                      potential at the atom), 385-256-192-160-1;
          "hcno_ee"-- as "hcno_mm" with a second output, a predicted atomic
                      charge q_i that enters as q_i phi_i, 385-256-192-160-2.
    """
    if kind == "water":
        species = (1, 8)
    elif kind in ("hcno", "hcno_mm", "hcno_ee"):
        species = (1, 6, 7, 8)
    else:
        raise ValueError(f"unknown model kind {kind!r}")
    S = len(species)
    D = 16 * S + 32 * (S * (S + 1) // 2)
    extra = 1 if kind in ("hcno_mm", "hcno_ee") else 0
    n_out = 2 if kind == "hcno_ee" else 1
    hidden = (160, 128, 96) if kind == "water" else (256, 192, 160)
    f32 = np.float32
    return {
        "kind": kind,
        "species": species,
        "rc_rad": f32(5.2),
        "rc_ang": f32(3.5),
        "eta_rad": f32(19.7),
        "eta_ang": f32(12.5),
        "zeta": f32(14.1),
        "rad_shift": np.linspace(0.9, 5.2, 16).astype(f32),
        "ang_shift": np.linspace(0.9, 3.5, 8).astype(f32),
        "ang_sect": ((2 * np.arange(4) + 1) * math.pi / 8).astype(f32),
        "widths": (D + extra,) + hidden + (n_out,),
        "celu_alpha": f32(0.1),
        "extra_inputs": extra,
        "mm_cutoff": f32(12.0),
        "ke_coulomb": KE_COULOMB,
    }


# --------------------------------------------------------------------------
# Counter-based weights: SplitMix64 (Steele, Lea & Flood 2014) + Box-Muller.
# --------------------------------------------------------------------------
_GAMMA = np.uint64(0x9E3779B97F4A7C15)
_M1 = np.uint64(0xBF58476D1CE4E5B9)
_M2 = np.uint64(0x94D049BB133111EB)


def splitmix64(seed: int, counter: np.ndarray) -> np.ndarray:
    """Output number ``counter`` (0-based) of the SplitMix64 stream started at ``seed``."""
    c = np.asarray(counter, dtype=np.uint64)
    with np.errstate(over="ignore"):
        z = np.uint64(seed & 0xFFFFFFFFFFFFFFFF) + (c + np.uint64(1)) * _GAMMA
        z = (z ^ (z >> np.uint64(30))) * _M1
        z = (z ^ (z >> np.uint64(27))) * _M2
        return z ^ (z >> np.uint64(31))


def uniform01(seed: int, counter: np.ndarray) -> np.ndarray:
    """Uniform doubles in [0, 1): the top 53 bits of each SplitMix64 output."""
    return (splitmix64(seed, counter) >> np.uint64(11)).astype(np.float64) * (2.0 ** -53)


def _normals(seed: int, start: int, n: int) -> np.ndarray:
    """n standard normals; normal t uses uniforms start+2t and start+2t+1.

    z = sqrt(-2 ln(1 - u0)) * cos(2 pi u1), evaluated with the C library's
    log/cos/sqrt (Python's math module) so a C implementation of the same
    definition reproduces every value.
    """
    u = uniform01(seed, np.arange(start, start + 2 * n, dtype=np.uint64))
    out = np.empty(n, dtype=np.float64)
    two_pi = 2.0 * math.pi
    for t in range(n):
        out[t] = math.sqrt(-2.0 * math.log(1.0 - u[2 * t])) * math.cos(two_pi * u[2 * t + 1])
    return out


def model_weights(cfg: dict, seed: int = 1, n_members: int = 1):
    """Xavier-normal weights for every (ensemble member, species, layer).

    Returns ``w[member][species] = [(W1, b1), ..., (W4, b4)]`` with W of shape
    (out, in), float32.  Draw order: member, species, layer, then W (row-major)
    then b; W ~ N(0, 2/(fan_in+fan_out)), b ~ N(0, 0.1^2).  Each value is
    rounded once to FP32.
    """
    widths = cfg["widths"]
    S = len(cfg["species"])
    counter = 0
    members = []
    for _m in range(n_members):
        per_species = []
        for _s in range(S):
            layers = []
            for l in range(len(widths) - 1):
                fi, fo = widths[l], widths[l + 1]
                std_w = math.sqrt(2.0 / (fi + fo))
                zw = _normals(seed, counter, fo * fi)
                counter += 2 * fo * fi
                zb = _normals(seed, counter, fo)
                counter += 2 * fo
                W = (zw * std_w).astype(np.float32).reshape(fo, fi)
                b = (zb * 0.1).astype(np.float32)
                layers.append((W, b))
            per_species.append(layers)
        members.append(per_species)
    return members


def flat_weights(w) -> np.ndarray:
    """Concatenate weights in draw order (member, species, layer, W row-major, b)."""
    parts = []
    for per_species in w:
        for layers in per_species:
            for W, b in layers:
                parts.append(W.reshape(-1))
                parts.append(b.reshape(-1))
    return np.concatenate(parts).astype(np.float32)


# --------------------------------------------------------------------------
# Geometries.
# --------------------------------------------------------------------------
def _quaternion_rotations(u: np.ndarray) -> np.ndarray:
    """Uniform random rotations from three uniforms per sample (Shoemake 1992)."""
    u1, u2, u3 = u[:, 0], u[:, 1], u[:, 2]
    a = np.sqrt(1.0 - u1)
    b = np.sqrt(u1)
    q0 = a * np.sin(2 * np.pi * u2)
    q1 = a * np.cos(2 * np.pi * u2)
    q2 = b * np.sin(2 * np.pi * u3)
    q3 = b * np.cos(2 * np.pi * u3)
    # (w, x, y, z) = (q3, q0, q1, q2)
    w, x, y, z = q3, q0, q1, q2
    R = np.empty((u.shape[0], 3, 3))
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


def water_box(n_mol: int, L: float, seed: int = 0, n_side: int | None = None,
              jitter: float = 0.3):
    """Periodic cubic water box.

    Oxygens sit at the centres of an n_side^3 lattice of spacing L/n_side (a
    seeded subset of sites when n_mol < n_side^3), jittered by U(-jitter,
    jitter) per component; each molecule gets a uniform random orientation.
    Coordinates are NOT wrapped into [0, L).  Atom order: O, H, H per molecule.
    Returns (pos float32 [3 n_mol, 3], Z int32 [3 n_mol], box float32 [3]).
    """
    rng = np.random.Generator(np.random.PCG64(seed))
    if n_side is None:
        n_side = int(round(n_mol ** (1.0 / 3.0)))
        while n_side ** 3 < n_mol:
            n_side += 1
    sites = n_side ** 3
    if sites < n_mol:
        raise ValueError("lattice too small")
    spacing = L / n_side
    if sites == n_mol:
        idx = np.arange(sites)
    else:
        idx = np.sort(rng.permutation(sites)[:n_mol])
    g = np.stack(np.unravel_index(idx, (n_side, n_side, n_side)), axis=1).astype(np.float64)
    O = (g + 0.5) * spacing + rng.uniform(-jitter, jitter, size=(n_mol, 3))
    R = _quaternion_rotations(rng.random((n_mol, 3)))
    half = 0.5 * _HOH
    local = np.array([[_OH * math.sin(half), 0.0, _OH * math.cos(half)],
                      [-_OH * math.sin(half), 0.0, _OH * math.cos(half)]])
    H = O[:, None, :] + np.einsum("nij,hj->nhi", R, local)
    pos = np.empty((n_mol, 3, 3))
    pos[:, 0] = O
    pos[:, 1:] = H
    Z = np.tile(np.array([8, 1, 1], dtype=np.int32), n_mol)
    box = np.full(3, L, dtype=np.float32)
    return pos.reshape(-1, 3).astype(np.float32), Z, box


def walk_molecule(n: int, rng: np.random.Generator, box: float = 40.0,
                  bond=(1.0, 1.5), dmin: float = 0.9, origin=None):
    """Self-avoiding random-walk molecule of n atoms (H/C/N/O 0.5/0.3/0.1/0.1).

    Starts at the box centre; each new atom sits U(bond) from the current
    anchor in a uniform direction; proposals closer than dmin to any atom or
    outside [0, box)^3 are rejected, and after 100 rejections in a row the
    anchor moves to a uniformly chosen earlier atom.
    Returns (pos float32 [n, 3], Z int32 [n]).
    """
    Z = rng.choice(np.array([1, 6, 7, 8], dtype=np.int32), size=n, p=[0.5, 0.3, 0.1, 0.1])
    pts = np.empty((n, 3))
    pts[0] = box / 2.0
    m = 1
    anchor = 0
    fails = 0
    d2min = dmin * dmin
    while m < n:
        v = rng.normal(size=3)
        v /= np.linalg.norm(v)
        p = pts[anchor] + rng.uniform(bond[0], bond[1]) * v
        ok = bool(np.all(p >= 0.0) and np.all(p < box))
        if ok:
            d2 = np.sum((pts[:m] - p) ** 2, axis=1)
            ok = bool(np.all(d2 >= d2min))
        if ok:
            pts[m] = p
            anchor = m
            m += 1
            fails = 0
        else:
            fails += 1
            if fails >= 100:
                anchor = int(rng.integers(0, m))
                fails = 0
    if origin is not None:
        pts = pts + np.asarray(origin, dtype=np.float64)
    return pts.astype(np.float32), Z


def walk_batch(n_mol: int = 256, seed: int = 0, nmin: int = 24, nmax: int = 300):
    """Uneven batch of walk molecules with sizes floor(exp(U(ln nmin, ln(nmax+1)))).

    Returns (pos float32 [sum n, 3], Z int32 [sum n], offsets int32 [n_mol+1]).
    """
    rng = np.random.Generator(np.random.PCG64(seed))
    sizes = np.floor(np.exp(rng.uniform(math.log(nmin), math.log(nmax + 1), size=n_mol))).astype(np.int64)
    sizes = np.clip(sizes, nmin, nmax)
    pos, Z = [], []
    for n in sizes:
        p, z = walk_molecule(int(n), rng)
        pos.append(p)
        Z.append(z)
    offsets = np.zeros(n_mol + 1, dtype=np.int32)
    offsets[1:] = np.cumsum(sizes)
    return np.concatenate(pos), np.concatenate(Z), offsets


def solute_in_water(seed: int = 0, n_solute: int = 60, n_side: int = 22, L: float = 68.3,
                    n_keep: int = 10000, clearance: float = 2.0):
    """A walk solute at the centre of a periodic box of fixed-charge MM water.

    The water box is built like ``water_box`` (n_side^3 sites); waters with
    any atom within ``clearance`` of a solute atom are dropped, then a seeded
    permutation keeps exactly n_keep waters.  Charges: O -0.834 e, H +0.417 e.
    Returns dict(pos, Z, mm_pos, mm_q, box).
    """
    rng = np.random.Generator(np.random.PCG64(seed + 1000))
    origin = (L - 40.0) / 2.0
    sp, sz = walk_molecule(n_solute, rng, box=40.0, origin=(origin, origin, origin))
    wp, wz, box = water_box(n_side ** 3, L, seed=seed)
    wp64 = wp.astype(np.float64).reshape(-1, 3, 3)
    d = wp64[:, :, None, :] - sp.astype(np.float64)[None, None, :, :]
    d -= L * np.rint(d / L)
    close = np.any(np.sum(d * d, axis=-1) < clearance * clearance, axis=(1, 2))
    keep = np.nonzero(~close)[0]
    if keep.size < n_keep:
        raise ValueError("not enough waters left")
    keep = np.sort(rng.permutation(keep)[:n_keep])
    mm_pos = wp.reshape(-1, 3, 3)[keep].reshape(-1, 3)
    mm_q = np.tile(np.array([-0.834, 0.417, 0.417], dtype=np.float32), n_keep)
    return {"pos": sp, "Z": sz, "mm_pos": np.ascontiguousarray(mm_pos), "mm_q": mm_q,
            "box": np.full(3, L, dtype=np.float32)}


# Lennard-Jones parameters (sigma A, epsilon eV) of the order of general
# force-field values per element, and TIP3P water (H carries no LJ site).
_LJ_ELEMENT = {1: (2.50, 0.0013), 6: (3.40, 0.0037), 7: (3.25, 0.0073), 8: (3.00, 0.0091)}
TIP3P = {"q": (-0.834, 0.417, 0.417), "sigma": (3.1507, 0.0, 0.0), "eps": (0.0065955, 0.0, 0.0)}


def lj_params_solute(Z: np.ndarray, seed: int = 4) -> np.ndarray:
    """[n, 3] float32 (q, sigma, eps) for a solute: element LJ values and seeded partial
    charges U(-0.6, 0.6) shifted to a neutral total."""
    rng = np.random.Generator(np.random.PCG64(seed))
    q = rng.uniform(-0.6, 0.6, len(Z))
    q -= q.mean()
    sig = np.array([_LJ_ELEMENT[int(z)][0] for z in Z])
    eps = np.array([_LJ_ELEMENT[int(z)][1] for z in Z])
    return np.ascontiguousarray(np.column_stack([q, sig, eps]).astype(np.float32))


def lj_params_water(n_waters: int) -> np.ndarray:
    """[3 n_waters, 3] float32 (q, sigma, eps) of TIP3P water in O, H, H order."""
    one = np.column_stack([TIP3P["q"], TIP3P["sigma"], TIP3P["eps"]])
    return np.ascontiguousarray(np.tile(one, (n_waters, 1)).astype(np.float32))


def maxwell_boltzmann(Z: np.ndarray, T: float = 300.0, seed: int = 2) -> np.ndarray:
    """Velocities (A/fs, float64) at exactly temperature T with 3N-3 degrees of freedom."""
    rng = np.random.Generator(np.random.PCG64(seed))
    m = np.array([WATER_MASS[int(z)] for z in Z], dtype=np.float64)
    sigma = np.sqrt(KB_EV * T / m * ACC_UNIT)        # A/fs
    v = rng.normal(size=(len(Z), 3)) * sigma[:, None]
    v -= (m[:, None] * v).sum(0) / m.sum()
    ke = 0.5 * np.sum(m[:, None] * v * v) / ACC_UNIT  # eV
    ke_target = 0.5 * (3 * len(Z) - 3) * KB_EV * T
    return v * math.sqrt(ke_target / ke)
