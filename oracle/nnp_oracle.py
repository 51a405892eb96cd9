"""Plain FP64 CPU oracle for the NNP energy + force path.

TEST INFRASTRUCTURE ONLY.  Only the test-suite, the smoke check and the CPU
baseline leg of the benchmark may import this module.  It shares no code with
the HIP library (no kernels, headers, tables or helpers) and imports nothing
from the product package; its inputs come from ``synthetic`` or from the
caller.

What it computes (everything in float64, inputs promoted from the exact FP32
values the GPU receives):

* the ML/MM force contract of the paper's Theory section: the NNP supplies
  E_ML for the atoms of an index group and the forces F_i = -grad_i E_ML
  (eq. 2); atoms outside the group get zero force.  The model inputs are the
  atomic numbers, positions, box and periodicity, optionally MM positions and
  charges (Methods, "The nnpot Interface");
* the ANI-family descriptor-based NNP that the paper runs and benchmarks
  (ANI2x through TorchANI / NNPOps, Methods and the performance section):
  radial and modified-angular symmetry functions feeding one MLP per element,
  E = sum_i e_i;
* the readings this build freezes where the paper is silent: closed shift
  grids, the 2^(1-zeta) angular prefactor, unordered (j < k) angular pairs,
  theta' = arccos(0.95 cos theta), species-pair order, CELU(alpha=0.1).

Forces come from torch.autograd in float64 (a library primitive used as the
differentiation step); the tests pin them with central finite differences.

Also here, as the plain definitions of the integer stages, are the FP32 cell
binning and neighbour predicates (``cell_list_fp32``, ``neighbours_fp32``),
written op by op in float32 so the GPU's integer outputs can be compared bit
for bit.
"""
from __future__ import annotations

import math

import numpy as np
import torch

__all__ = [
    "species_index", "pair_class_table", "neighbour_pairs", "neighbour_pairs_bruteforce",
    "cutoff", "celu", "descriptors", "mlp_outputs", "mlp_energies", "mlp_input_grad", "evaluate",
    "evaluate_batch", "cell_list_fp32", "neighbours_fp32", "neighbours_fp32_kdtree", "mm_potential",
    "link_atom_positions",
    "me_coupling",
]

_F32 = np.float32


# --------------------------------------------------------------------------
# Species and species-pair indexing (frozen reading: ascending atomic number;
# unordered pairs a <= b in lexicographic order).
# --------------------------------------------------------------------------
def species_index(Z, species) -> np.ndarray:
    """sigma(Z): position of each atomic number in the ascending species table."""
    Z = np.asarray(Z)
    table = {int(z): k for k, z in enumerate(species)}
    out = np.empty(Z.shape, dtype=np.int64)
    for t, z in enumerate(Z.reshape(-1)):
        if int(z) not in table:
            raise ValueError(f"atomic number {int(z)} is not in the species table {tuple(species)}")
        out.reshape(-1)[t] = table[int(z)]
    return out


def pair_class_table(S: int) -> np.ndarray:
    """P[a, b] = index of the unordered species pair {a, b}, lexicographic with a <= b."""
    P = np.full((S, S), -1, dtype=np.int64)
    p = 0
    for a in range(S):
        for b in range(a, S):
            P[a, b] = p
            P[b, a] = p
            p += 1
    return P


# --------------------------------------------------------------------------
# Neighbours (float64 geometry).
# --------------------------------------------------------------------------
def _min_image_np(d, box):
    if box is None:
        return d
    L = np.asarray(box, dtype=np.float64)
    return d - L * np.rint(d / L)


def neighbour_pairs_bruteforce(pos, rc, box=None, centres=None):
    """All directed pairs (i, j), i != j, with |d_ij| < rc under the minimum image.

    O(N^2) in float64.  ``centres`` restricts i.  Returns (i, j) int64 arrays
    sorted by i then j.
    """
    pos = np.asarray(pos, dtype=np.float64)
    n = pos.shape[0]
    cs = np.arange(n) if centres is None else np.asarray(centres, dtype=np.int64)
    I, J = [], []
    for s in range(0, cs.size, 512):
        c = cs[s:s + 512]
        d = _min_image_np(pos[None, :, :] - pos[c, None, :], box)
        r2 = np.sum(d * d, axis=-1)
        ii, jj = np.nonzero(r2 < rc * rc)
        keep = c[ii] != jj
        I.append(c[ii][keep])
        J.append(jj[keep])
    I = np.concatenate(I) if I else np.zeros(0, np.int64)
    J = np.concatenate(J) if J else np.zeros(0, np.int64)
    o = np.lexsort((J, I))
    return I[o], J[o]


def neighbour_pairs(pos, rc, box=None, centres=None):
    """Same pair set as ``neighbour_pairs_bruteforce`` via a k-d tree (large N).

    Candidates come from scipy's cKDTree with a slightly larger radius, and
    the strict float64 predicate |d| < rc decides.
    """
    from scipy.spatial import cKDTree
    pos = np.asarray(pos, dtype=np.float64)
    n = pos.shape[0]
    if n == 0:
        return np.zeros(0, np.int64), np.zeros(0, np.int64)
    if box is not None:
        L = np.asarray(box, dtype=np.float64)
        wrapped = pos - L * np.floor(pos / L)
        wrapped = np.where(wrapped >= L, wrapped - L, wrapped)
        wrapped = np.where(wrapped < 0, 0.0, wrapped)
        tree = cKDTree(wrapped, boxsize=L)
        q = wrapped
    else:
        tree = cKDTree(pos)
        q = pos
    cs = np.arange(n) if centres is None else np.asarray(centres, dtype=np.int64)
    lists = tree.query_ball_point(q[cs], r=float(rc) + 1e-6)
    cnt = np.array([len(l) for l in lists], dtype=np.int64)
    I = np.repeat(cs, cnt)
    J = np.concatenate([np.asarray(l, dtype=np.int64) for l in lists]) if cnt.sum() else np.zeros(0, np.int64)
    d = _min_image_np(pos[J] - pos[I], box)
    keep = (np.sum(d * d, axis=1) < rc * rc) & (I != J)
    I, J = I[keep], J[keep]
    o = np.lexsort((J, I))
    return I[o], J[o]


# --------------------------------------------------------------------------
# Elementary functions of the model (torch float64, differentiable).
# --------------------------------------------------------------------------
def cutoff(r, rc):
    """fc(r) = 0.5 cos(pi r / rc) + 0.5 for r < rc, else 0."""
    inside = r < rc
    val = 0.5 * torch.cos(math.pi * r / rc) + 0.5
    return torch.where(inside, val, torch.zeros_like(val))


def celu(u, alpha):
    """CELU_alpha(u) = max(0, u) + min(0, alpha (exp(u/alpha) - 1)).

    The second term vanishes for u >= 0, so its exponent is taken at min(u, 0):
    the same function, without exp overflowing (and its gradient turning NaN)
    for large positive u."""
    return torch.clamp(u, min=0.0) + torch.clamp(alpha * torch.expm1(torch.clamp(u, max=0.0) / alpha), max=0.0)


def _min_image_t(d, box_t):
    if box_t is None:
        return d
    return d - box_t * torch.round(d / box_t)   # torch.round rounds half to even


def _triplet_index(ci_sorted):
    """For pairs grouped by centre (ci non-decreasing), all index pairs (a, b) with
    a < b inside each centre's group.  Returns (a_idx, b_idx) into the pair arrays."""
    if ci_sorted.size == 0:
        return np.zeros(0, np.int64), np.zeros(0, np.int64)
    uniq, starts, counts = np.unique(ci_sorted, return_index=True, return_counts=True)
    npair = counts * (counts - 1) // 2
    M = int(counts.max())
    # enumerate (a, b), a < b < M, ordered by b then a: the first n(n-1)/2
    # entries are exactly the pairs of a group of n.
    bb = np.repeat(np.arange(M), np.arange(M))
    aa = np.concatenate([np.arange(b) for b in range(M)]) if M > 1 else np.zeros(0, np.int64)
    total = int(npair.sum())
    grp = np.repeat(np.arange(uniq.size), npair)
    local = np.arange(total) - np.repeat(np.cumsum(npair) - npair, npair)
    return starts[grp] + aa[local], starts[grp] + bb[local]


# --------------------------------------------------------------------------
# Descriptors.
# --------------------------------------------------------------------------
def descriptors(pos_t, sigma, cfg, box=None, centres=None, pairs_rad=None, mm=None):
    """ANI-style atomic environment vectors for the centre atoms, float64.

    pos_t  : torch float64 [n, 3] (may require grad)
    sigma  : int species index per atom [n]
    cfg    : hyper-parameters (see synthetic.model_config)
    centres: atoms whose descriptors are wanted (default: all)
    pairs_rad: optional precomputed directed radial pairs (i, j) restricted to centres
    mm     : optional (mm_pos_t [m, 3] float64, mm_q [m] float64) for the extra
             input channel phi_i (appended as the last column)

    Layout of one row: radial block [species s][shift k] (16 per species), then
    angular block [species pair p][radial shift m][angle section n] (8 x 4 per pair).
    """
    n = pos_t.shape[0]
    S = len(cfg["species"])
    nR = len(cfg["rad_shift"])
    nAm = len(cfg["ang_shift"])
    nAn = len(cfg["ang_sect"])
    P = S * (S + 1) // 2
    D = S * nR + P * nAm * nAn
    cs = np.arange(n) if centres is None else np.asarray(centres, dtype=np.int64)
    row_of = -np.ones(n, dtype=np.int64)
    row_of[cs] = np.arange(cs.size)
    rc = float(cfg["rc_rad"])
    rca = float(cfg["rc_ang"])
    eta_r = float(cfg["eta_rad"])
    eta_a = float(cfg["eta_ang"])
    zeta = float(cfg["zeta"])
    rs = torch.tensor(np.asarray(cfg["rad_shift"], np.float64))
    ras = torch.tensor(np.asarray(cfg["ang_shift"], np.float64))
    th = torch.tensor(np.asarray(cfg["ang_sect"], np.float64))
    box_t = None if box is None else torch.tensor(np.asarray(box, np.float64))
    sigma = np.asarray(sigma, dtype=np.int64)

    if pairs_rad is None:
        pos_np = pos_t.detach().numpy()
        I, J = neighbour_pairs(pos_np, rc, box, centres=cs)
    else:
        I, J = pairs_rad
    x = torch.zeros((cs.size, D), dtype=torch.float64)

    # radial: G[i, s, k] = sum_{j: sigma_j = s} exp(-eta (r - Rs_k)^2) fc(r; Rc)
    d = _min_image_t(pos_t[J] - pos_t[I], box_t)
    r = torch.sqrt(torch.sum(d * d, dim=1))
    g = torch.exp(-eta_r * (r[:, None] - rs[None, :]) ** 2) * cutoff(r, rc)[:, None]
    cols = torch.tensor(sigma[J] * nR)[:, None] + torch.arange(nR)[None, :]
    rows = torch.tensor(row_of[I])[:, None].expand(-1, nR)
    x = x.index_put((rows.reshape(-1), cols.reshape(-1)), g.reshape(-1), accumulate=True)

    # angular: unordered neighbour pairs (j, k), both within Rc_a of i
    ang = (r < rca).detach().numpy()
    Ia, Ja = I[ang], J[ang]
    da = d[torch.tensor(np.nonzero(ang)[0])]
    ra = r[torch.tensor(np.nonzero(ang)[0])]
    a_idx, b_idx = _triplet_index(Ia)
    if a_idx.size:
        at = torch.tensor(a_idx)
        bt = torch.tensor(b_idx)
        dj, dk = da[at], da[bt]
        rj, rk = ra[at], ra[bt]
        cos_t = torch.sum(dj * dk, dim=1) / (rj * rk)
        theta = torch.arccos(0.95 * cos_t)
        rbar = 0.5 * (rj + rk)
        fcj = cutoff(rj, rca)
        fck = cutoff(rk, rca)
        ang_part = (1.0 + torch.cos(theta[:, None] - th[None, :])) ** zeta        # [T, nAn]
        rad_part = torch.exp(-eta_a * (rbar[:, None] - ras[None, :]) ** 2)        # [T, nAm]
        pref = (2.0 ** (1.0 - zeta)) * fcj * fck
        terms = pref[:, None, None] * rad_part[:, :, None] * ang_part[:, None, :]  # [T, nAm, nAn]
        ptab = pair_class_table(S)
        p = ptab[sigma[Ja[a_idx]], sigma[Ja[b_idx]]]
        base = S * nR + p * (nAm * nAn)
        cols = torch.tensor(base)[:, None] + torch.arange(nAm * nAn)[None, :]
        rows = torch.tensor(row_of[Ia[a_idx]])[:, None].expand(-1, nAm * nAn)
        x = x.index_put((rows.reshape(-1), cols.reshape(-1)), terms.reshape(terms.shape[0], -1).reshape(-1),
                        accumulate=True)

    if mm is not None:
        mm_pos_t, mm_q = mm
        phi = mm_potential(pos_t[torch.tensor(cs)], mm_pos_t, mm_q, cfg, box)
        x = torch.cat([x, phi[:, None]], dim=1)
    return x


def mm_potential(pos_c, mm_pos_t, mm_q, cfg, box=None):
    """phi_i = k_e sum_j q_j fc(r_ij; R_mm) / r_ij over MM atoms j (minimum image)."""
    Rm = float(cfg["mm_cutoff"])
    ke = float(cfg["ke_coulomb"])
    q = torch.as_tensor(np.asarray(mm_q, np.float64))
    box_t = None if box is None else torch.tensor(np.asarray(box, np.float64))
    out = []
    for s in range(0, pos_c.shape[0], 64):
        d = _min_image_t(mm_pos_t[None, :, :] - pos_c[s:s + 64, None, :], box_t)
        r = torch.sqrt(torch.sum(d * d, dim=-1))
        inside = r < Rm
        rsafe = torch.where(inside, r, torch.ones_like(r))
        term = torch.where(inside, q[None, :] * cutoff(rsafe, Rm) / rsafe, torch.zeros_like(r))
        out.append(ke * term.sum(dim=1))
    return torch.cat(out) if out else torch.zeros(0, dtype=torch.float64)


# --------------------------------------------------------------------------
# Per-element networks.
# --------------------------------------------------------------------------
def _as_t(a):
    return torch.as_tensor(np.asarray(a, np.float64))


def mlp_outputs(x, sigma_c, weights, alpha):
    """[rows, n_out] = W4 h3 + b4 with h_l = CELU(W_l h_{l-1} + b_l), one network per species."""
    n_out = len(weights[0][-1][1])
    o = torch.zeros((x.shape[0], n_out), dtype=torch.float64)
    sigma_c = np.asarray(sigma_c)
    for s, layers in enumerate(weights):
        rows = np.nonzero(sigma_c == s)[0]
        if rows.size == 0:
            continue
        h = x[torch.tensor(rows)]
        for l, (W, b) in enumerate(layers):
            h = h @ _as_t(W).T + _as_t(b)
            if l < len(layers) - 1:
                h = celu(h, float(alpha))
        o = o.index_put((torch.tensor(rows),), h)
    return o


def mlp_energies(x, sigma_c, weights, alpha):
    """Atomic energies.  One output: e_i.  Two outputs (models with the MM
    potential as last input): the second is a predicted atomic charge q_i in
    the MM potential phi_i, e_i + q_i phi_i -- electrostatic embedding with
    charges from the model (Methods: the model may return charges / put
    forces on MM atoms)."""
    o = mlp_outputs(x, sigma_c, weights, alpha)
    if o.shape[1] == 1:
        return o[:, 0]
    return o[:, 0] + o[:, 1] * x[:, -1]


def mlp_input_grad(x_np, sigma_c, weights, alpha):
    """d e_i / d x_i for every row (float64), via autograd through ``mlp_energies``."""
    x = torch.tensor(np.asarray(x_np, np.float64), requires_grad=True)
    e = mlp_energies(x, sigma_c, weights, alpha)
    (g,) = torch.autograd.grad(e.sum(), x)
    return e.detach().numpy(), g.numpy()


# --------------------------------------------------------------------------
# Energy and forces.
# --------------------------------------------------------------------------
def evaluate(pos, Z, cfg, weights, box=None, nnp_idx=None, mm_pos=None, mm_q=None,
             centres=None, chunk=2048, forces=True, return_x=False, links=None):
    """E_ML and F = -grad E_ML for the NNP atoms of one system (float64).

    pos      : [n, 3] positions (float32 values; promoted exactly)
    Z        : [n] atomic numbers
    weights  : model_weights(...) -- a list of ensemble members, each a list per
               species of [(W, b), ...]; the energy is the member average
    box      : [3] orthorhombic box lengths, or None for no periodicity
    nnp_idx  : indices of the NNP atoms (the index group); default all
    mm_pos/mm_q : MM point charges for the extra input channel (needs
               cfg["extra_inputs"] == 1)
    centres  : optional subset of NNP-local atom indices whose atomic
               energies are summed (E and the gradient then cover only those);
               used to get exact forces on sampled atoms of very large systems.
    links    : optional (ml_idx, mm_idx, d, Z_link): link atoms placed by eq. 4
               on the bonds ml -> mm (ml in the index group, mm outside; the
               bond vector under the minimum image when ``box`` is given); they
               are NNP atoms appended after the index group, and their forces
               reach the ML and MM atoms through the chain rule (autograd
               through the link positions).
    Returns dict(E, e [centres], F [n, 3], F_mm [m, 3] or None, x (optional)).
    """
    pos = np.asarray(pos)
    n = pos.shape[0]
    idx = np.arange(n) if nnp_idx is None else np.asarray(nnp_idx, dtype=np.int64)
    sigma = species_index(np.asarray(Z)[idx], cfg["species"])
    full = torch.tensor(pos.astype(np.float64), requires_grad=forces)
    if links is not None:
        ml, mmi, d_link, z_link = links
        ml = np.asarray(ml, dtype=np.int64)
        mmi = np.asarray(mmi, dtype=np.int64)
        sigma = np.concatenate([sigma, species_index(np.full(ml.size, z_link), cfg["species"])])

    def nnp_positions():
        p = full[torch.tensor(idx)]
        if links is not None and ml.size:
            rl = link_atom_positions(full[torch.tensor(ml)], full[torch.tensor(mmi)], float(d_link), box)
            p = torch.cat([p, rl])
        return p

    mm = None
    if cfg.get("extra_inputs", 0):
        if mm_pos is None:
            raise ValueError("this model needs MM positions and charges")
        mm_t = torch.tensor(np.asarray(mm_pos).astype(np.float64), requires_grad=forces)
        mm = (mm_t, np.asarray(mm_q, np.float64))
    members = weights if isinstance(weights[0][0], list) else [weights]
    n_nnp = sigma.size
    cs_all = np.arange(n_nnp) if centres is None else np.asarray(centres, dtype=np.int64)
    I, J = neighbour_pairs(nnp_positions().detach().numpy(), float(cfg["rc_rad"]), box, centres=cs_all)
    e_all = np.zeros(cs_all.size)
    xs = []
    grad = torch.zeros_like(full) if forces else None
    grad_mm = torch.zeros_like(mm[0]) if (forces and mm is not None) else None
    starts = np.searchsorted(I, cs_all)        # pairs are sorted by centre
    ends = np.searchsorted(I, cs_all, side="right")
    for s in range(0, cs_all.size, chunk):
        c = cs_all[s:s + chunk]
        lo, hi = starts[s], ends[min(s + chunk, cs_all.size) - 1]
        pr = (I[lo:hi], J[lo:hi])
        x = descriptors(nnp_positions(), sigma, cfg, box=box, centres=c, pairs_rad=pr, mm=mm)
        e = torch.zeros(c.size, dtype=torch.float64)
        for w in members:
            e = e + mlp_energies(x, sigma[c], w, cfg["celu_alpha"])
        e = e / len(members)
        e_all[s:s + c.size] = e.detach().numpy()
        if return_x:
            xs.append(x.detach().numpy())
        if forces:
            targets = [full] + ([mm[0]] if mm is not None else [])
            gs = torch.autograd.grad(e.sum(), targets, allow_unused=True)
            if gs[0] is not None:
                grad += gs[0]
            if mm is not None and gs[1] is not None:
                grad_mm += gs[1]
    out = {"E": math.fsum(e_all.tolist()), "e": e_all}
    if forces:
        out["F"] = -grad.numpy()
        out["F_mm"] = (-grad_mm.numpy()) if grad_mm is not None else None
    if return_x:
        out["x"] = np.concatenate(xs) if xs else np.zeros((0, 0))
    return out


def evaluate_batch(pos, Z, offsets, cfg, weights, forces=True, boxes=None):
    """Independent systems packed back to back: per-system E and all forces.

    boxes: None (every system open), or [n_sys][3] orthorhombic box lengths per
    system, a row of zeros (or NaN) marking an open system."""
    offsets = np.asarray(offsets)
    E = np.zeros(offsets.size - 1)
    F = np.zeros((pos.shape[0], 3))
    for m in range(offsets.size - 1):
        a, b = int(offsets[m]), int(offsets[m + 1])
        box = None
        if boxes is not None:
            row = np.asarray(boxes[m], np.float64)
            if np.all(np.isfinite(row)) and np.all(row > 0):
                box = row
        r = evaluate(pos[a:b], Z[a:b], cfg, weights, box=box, forces=forces)
        E[m] = r["E"]
        if forces:
            F[a:b] = r["F"]
    return E, F


# --------------------------------------------------------------------------
# Link atoms (eq. 4): r_L = r_ML + d (r_MM - r_ML) / |r_MM - r_ML|.
# --------------------------------------------------------------------------
def link_atom_positions(r_ml, r_mm, d=1.0, box=None):
    """Positions of link atoms placed at distance d from the ML atom along the ML-MM bond.

    In a periodic box the bond is the shortest one between the two atoms: u is
    taken under the minimum image, u - L round(u / L) per component (a bond is
    far shorter than half a box length, so this is the bonded copy of the MM
    atom whichever images the caller's coordinates hold)."""
    r_ml = torch.as_tensor(r_ml, dtype=torch.float64)
    r_mm = torch.as_tensor(r_mm, dtype=torch.float64)
    u = r_mm - r_ml
    if box is not None:
        u = _min_image_t(u, torch.tensor(np.asarray(box, np.float64)))
    return r_ml + d * u / torch.sqrt(torch.sum(u * u, dim=-1, keepdim=True))


# --------------------------------------------------------------------------
# Mechanical embedding (Theory, eq. 3): the ML-MM coupling stays at the MM
# level -- Coulomb plus Lennard-Jones between every ML atom and every MM atom,
# with fixed force-field charges and LJ parameters.  Readings: Lorentz-
# Berthelot mixing (the rule of the GAFF and CHARMM force fields used in the
# paper's Methods), a plain spherical cutoff without shift, minimum image.
# --------------------------------------------------------------------------
def me_coupling(ml_pos, ml_param, mm_pos, mm_param, ke, box=None, cutoff=None, forces=True, return_abs=False):
    """E = sum_{i in ML} sum_{j in MM, r_ij < cutoff} ke q_i q_j / r_ij
                                      + 4 eps_ij ((s_ij / r_ij)^12 - (s_ij / r_ij)^6),
    s_ij = (s_i + s_j) / 2, eps_ij = sqrt(eps_i eps_j); param rows are (q, sigma, eps).
    cutoff None takes every pair.  Returns (E, F_ml, F_mm) in float64 (forces by
    autograd, F = -dE/dr), and with return_abs also sum_ij |pair energy|."""
    x = torch.tensor(np.asarray(ml_pos, np.float64), requires_grad=forces)
    y = torch.tensor(np.asarray(mm_pos, np.float64), requires_grad=forces)
    pi = torch.as_tensor(np.asarray(ml_param, np.float64))
    pj = torch.as_tensor(np.asarray(mm_param, np.float64))
    d = y[None, :, :] - x[:, None, :]
    if box is not None:
        L = torch.as_tensor(np.asarray(box, np.float64))
        d = d - L * torch.round(d / L)
    r = torch.sqrt(torch.sum(d * d, dim=-1))
    qq = pi[:, None, 0] * pj[None, :, 0]
    sig = 0.5 * (pi[:, None, 1] + pj[None, :, 1])
    eps = torch.sqrt(pi[:, None, 2] * pj[None, :, 2])
    sr6 = (sig / r) ** 6
    pair = ke * qq / r + 4.0 * eps * (sr6 * sr6 - sr6)
    if cutoff is not None:
        pair = torch.where(r < cutoff, pair, torch.zeros_like(pair))
    E = pair.sum()
    F_ml = F_mm = None
    if forces:
        gx, gy = torch.autograd.grad(E, (x, y))
        F_ml, F_mm = (-gx).numpy(), (-gy).numpy()
    out = (float(E.detach()), F_ml, F_mm)
    if return_abs:
        out = out + (float(pair.detach().abs().sum()),)
    return out


# --------------------------------------------------------------------------
# Integer stages, defined op by op in IEEE float32 (no fused multiply-add).
# --------------------------------------------------------------------------
def _cells_per_dim(box32, rc32):
    return np.maximum(1, np.floor(box32 / rc32).astype(np.int64))


def cell_list_fp32(pos32, sigma, n_species, box32, rc32):
    """Cell binning and the stable counting sort by key = species * n_cells + cell.

    Per dimension: n_c = max(1, floor(L / rc)); invL = 1 / L; t = x * invL;
    w = x - floor(t) * L (wrap for binning only); c = floor(w * (n_c * invL))
    clamped to [0, n_c - 1].  Cell id = (cx * n_cy + cy) * n_cz + cz.
    Returns dict(n_c [3], cell [n], key [n], perm [n] (sorted slot -> atom),
    bin_start [n_species * n_cells + 1]).
    """
    pos32 = np.asarray(pos32, dtype=_F32)
    box32 = np.asarray(box32, dtype=_F32)
    rc32 = _F32(rc32)
    nc = _cells_per_dim(box32, rc32)
    inv = (_F32(1.0) / box32).astype(_F32)
    scale = (nc.astype(_F32) * inv).astype(_F32)
    c = np.empty(pos32.shape, dtype=np.int64)
    for k in range(3):
        x = pos32[:, k]
        t = (x * inv[k]).astype(_F32)
        w = (x - (np.floor(t).astype(_F32) * box32[k]).astype(_F32)).astype(_F32)
        ck = np.floor((w * scale[k]).astype(_F32)).astype(np.int64)
        c[:, k] = np.clip(ck, 0, nc[k] - 1)
    cell = (c[:, 0] * nc[1] + c[:, 1]) * nc[2] + c[:, 2]
    ncell = int(nc.prod())
    key = np.asarray(sigma, np.int64) * ncell + cell
    perm = np.argsort(key, kind="stable")
    hist = np.bincount(key, minlength=n_species * ncell)
    bin_start = np.zeros(n_species * ncell + 1, dtype=np.int64)
    bin_start[1:] = np.cumsum(hist)
    return {"n_c": nc, "cell": cell, "key": key, "perm": perm, "bin_start": bin_start}


def neighbours_fp32(pos32, rc32, box32=None):
    """Directed pairs (i, j), i != j, with r2 < rc*rc evaluated in float32:

    d = x_j - x_i; with a box, d = d - L * rint(d * (1/L)); r2 = (dx*dx + dy*dy) + dz*dz,
    every operation rounded to float32 (no fused multiply-add).
    Returns (i, j) sorted by i then j.
    """
    pos32 = np.asarray(pos32, dtype=_F32)
    n = pos32.shape[0]
    rc2 = _F32(_F32(rc32) * _F32(rc32))
    if box32 is not None:
        box32 = np.asarray(box32, dtype=_F32)
        inv = (_F32(1.0) / box32).astype(_F32)
    I, J = [], []
    for s in range(0, n, 256):
        c = np.arange(s, min(n, s + 256))
        d = (pos32[None, :, :] - pos32[c, None, :]).astype(_F32)
        if box32 is not None:
            sh = np.rint((d * inv).astype(_F32)).astype(_F32)
            d = (d - (sh * box32).astype(_F32)).astype(_F32)
        sq = (d * d).astype(_F32)
        r2 = ((sq[..., 0] + sq[..., 1]).astype(_F32) + sq[..., 2]).astype(_F32)
        ii, jj = np.nonzero(r2 < rc2)
        keep = c[ii] != jj
        I.append(c[ii][keep])
        J.append(jj[keep])
    I = np.concatenate(I) if I else np.zeros(0, np.int64)
    J = np.concatenate(J) if J else np.zeros(0, np.int64)
    o = np.lexsort((J, I))
    return I[o].astype(np.int64), J[o].astype(np.int64)


def _fp32_pair_r2(pos32, I, J, box32):
    """r2 of the directed pairs (I, J) by the float32 operations of ``neighbours_fp32``."""
    d = (pos32[J] - pos32[I]).astype(_F32)
    if box32 is not None:
        inv = (_F32(1.0) / box32).astype(_F32)
        sh = np.rint((d * inv).astype(_F32)).astype(_F32)
        d = (d - (sh * box32).astype(_F32)).astype(_F32)
    sq = (d * d).astype(_F32)
    return ((sq[:, 0] + sq[:, 1]).astype(_F32) + sq[:, 2]).astype(_F32)


def neighbours_fp32_kdtree(pos32, rc32, box32=None, margin=0.01):
    """The pair set of ``neighbours_fp32`` for systems too large for its O(N^2) scan.

    Candidates are the pairs a k-d tree (scipy cKDTree, float64 geometry of the
    same FP32 coordinates, periodic with ``boxsize`` when a box is given) finds
    within rc + margin; the float32 predicate of ``neighbours_fp32`` then decides
    each candidate in both directions.  The margin (0.01 A) is far above the
    float32 rounding of a displacement, so no pair the predicate accepts is
    missed.  Returns (i, j) sorted by i then j.
    """
    from scipy.spatial import cKDTree
    pos32 = np.asarray(pos32, dtype=_F32)
    n = pos32.shape[0]
    if n < 2:
        return np.zeros(0, np.int64), np.zeros(0, np.int64)
    p64 = pos32.astype(np.float64)
    if box32 is not None:
        box32 = np.asarray(box32, dtype=_F32)
        L = box32.astype(np.float64)
        w = p64 - L * np.floor(p64 / L)
        w = np.where(w >= L, w - L, w)
        w = np.where(w < 0, 0.0, w)
        tree = cKDTree(w, boxsize=L)
    else:
        tree = cKDTree(p64)
    pr = tree.query_pairs(r=float(rc32) + margin, output_type="ndarray").astype(np.int64)
    I = np.concatenate([pr[:, 0], pr[:, 1]])
    J = np.concatenate([pr[:, 1], pr[:, 0]])
    rc2 = _F32(_F32(rc32) * _F32(rc32))
    keep = _fp32_pair_r2(pos32, I, J, box32) < rc2
    I, J = I[keep], J[keep]
    o = np.lexsort((J, I))
    return I[o], J[o]
