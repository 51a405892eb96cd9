"""Pins for the FP64 oracle: closed forms, library routines, invariants, finite
differences, brute force.  CPU only.

None of these re-run the oracle's own formulas on the oracle's own output:
the closed forms are evaluated independently in 30-digit mpmath for special
geometries, the network is compared with torch.nn building blocks, and forces
with central finite differences of the energy.
"""
import math

import mpmath
import numpy as np
import pytest
import torch

import oracle as orc
import synthetic as sy

mpmath.mp.dps = 30
WATER = sy.model_config("water")
HCNO = sy.model_config("hcno")
HCNO_MM = sy.model_config("hcno_mm")
HCNO_EE = sy.model_config("hcno_ee")


@pytest.fixture(scope="module")
def w_water():
    return sy.model_weights(WATER, seed=1)


@pytest.fixture(scope="module")
def w_hcno():
    return sy.model_weights(HCNO, seed=1)


@pytest.fixture(scope="module")
def box64():
    return sy.water_box(64, 12.42, seed=0)


# ---------------------------------------------------------------- closed forms
def _mp(v):
    return mpmath.mpf(float(v))


def mp_fc(r, rc):
    return mpmath.mpf("0.5") * mpmath.cos(mpmath.pi * r / rc) + mpmath.mpf("0.5") if r < rc else mpmath.mpf(0)


def mp_radial(r, cfg):
    eta, rc = _mp(cfg["eta_rad"]), _mp(cfg["rc_rad"])
    return [mpmath.e ** (-eta * (r - _mp(s)) ** 2) * mp_fc(r, rc) for s in cfg["rad_shift"]]


def mp_angular(dj, dk, cfg):
    """8 x 4 modified-angular terms of one (j, k) pair seen from the centre."""
    rj = mpmath.sqrt(sum(a * a for a in dj))
    rk = mpmath.sqrt(sum(a * a for a in dk))
    cos_t = sum(a * b for a, b in zip(dj, dk)) / (rj * rk)
    th = mpmath.acos(mpmath.mpf("0.95") * cos_t)
    zeta, eta, rca = _mp(cfg["zeta"]), _mp(cfg["eta_ang"]), _mp(cfg["rc_ang"])
    rbar = (rj + rk) / 2
    pref = mpmath.mpf(2) ** (1 - zeta) * mp_fc(rj, rca) * mp_fc(rk, rca)
    out = []
    for m in cfg["ang_shift"]:
        for n in cfg["ang_sect"]:
            out.append(pref * (1 + mpmath.cos(th - _mp(n))) ** zeta * mpmath.e ** (-eta * (rbar - _mp(m)) ** 2))
    return out


def _mpvec(p):
    return [mpmath.mpf(float(v)) for v in p]


def _sub(a, b):
    return [x - y for x, y in zip(a, b)]


def test_radial_dimer_closed_form(w_water):
    # H at the origin, O at distance ~1.07 along a skew direction
    pos = np.array([[0.0, 0.0, 0.0], [0.9, 0.4, -0.45]])
    Z = np.array([1, 8])
    x = orc.evaluate(pos, Z, WATER, w_water, box=None, forces=False, return_x=True)["x"]
    r = mpmath.sqrt(sum(_mp(v) ** 2 for v in pos[1]))
    g = [float(v) for v in mp_radial(r, WATER)]
    ref_H = np.zeros(128)
    ref_H[16:32] = g          # H-centred: neighbour is O (species 1)
    ref_O = np.zeros(128)
    ref_O[0:16] = g           # O-centred: neighbour is H (species 0)
    np.testing.assert_allclose(x[0], ref_H, rtol=1e-13, atol=1e-300)
    np.testing.assert_allclose(x[1], ref_O, rtol=1e-13, atol=1e-300)


def _water_monomer():
    half = math.radians(104.52) / 2
    oh = 0.9572
    return np.array([[0.0, 0.0, 0.0],
                     [oh * math.sin(half), 0.0, oh * math.cos(half)],
                     [-oh * math.sin(half), 0.0, oh * math.cos(half)]]), np.array([8, 1, 1])


def test_single_water_full_descriptor_closed_form(w_water):
    pos, Z = _water_monomer()
    x = orc.evaluate(pos, Z, WATER, w_water, box=None, forces=False, return_x=True)["x"]
    P = [_mpvec(p) for p in pos]
    ref = np.zeros((3, 128))
    # O-centred: two H neighbours, one (H, H) angular pair (class HH = 0)
    dO1, dO2 = _sub(P[1], P[0]), _sub(P[2], P[0])
    rO1 = mpmath.sqrt(sum(a * a for a in dO1))
    rO2 = mpmath.sqrt(sum(a * a for a in dO2))
    ref[0, 0:16] = [float(a + b) for a, b in zip(mp_radial(rO1, WATER), mp_radial(rO2, WATER))]
    ref[0, 32:64] = [float(v) for v in mp_angular(dO1, dO2, WATER)]
    # H-centred: O and the other H as neighbours; one (H, O) pair, class HO = 1
    for c, other in ((1, 2), (2, 1)):
        dO = _sub(P[0], P[c])
        dH = _sub(P[other], P[c])
        rO = mpmath.sqrt(sum(a * a for a in dO))
        rH = mpmath.sqrt(sum(a * a for a in dH))
        ref[c, 0:16] = [float(v) for v in mp_radial(rH, WATER)]
        ref[c, 16:32] = [float(v) for v in mp_radial(rO, WATER)]
        ref[c, 64:96] = [float(v) for v in mp_angular(dH, dO, WATER)]
    np.testing.assert_allclose(x, ref, rtol=1e-12, atol=1e-300)
    # the O-centred (H,H) block peaks in the section containing 104.52 deg:
    # sections are centred at 22.5, 67.5, 112.5, 157.5 deg
    blk = x[0, 32:64].reshape(8, 4)
    assert np.argmax(blk[0]) == 2


def test_angular_term_at_section_centre():
    # closed form: (1 + cos 0)^zeta * 2^(1-zeta) = 2 when theta' equals a section centre
    cfg = dict(WATER)
    th_n = float(cfg["ang_sect"][1])
    cos_t = math.cos(th_n) / 0.95   # then arccos(0.95 cos_t) = th_n
    r = 1.2
    dj = [mpmath.mpf(r), 0, 0]
    dk = [r * mpmath.mpf(cos_t), r * mpmath.sqrt(1 - mpmath.mpf(cos_t) ** 2), 0]
    terms = mp_angular(dj, dk, cfg)
    pos = np.array([[0, 0, 0], [r, 0, 0], [r * cos_t, r * math.sqrt(1 - cos_t ** 2), 0.0]])
    x = orc.descriptors(torch.tensor(pos), np.array([0, 0, 0]), cfg)
    fc = float(mp_fc(mpmath.mpf(r), _mp(cfg["rc_ang"]))) ** 2
    ang = x[0, 32:64].numpy().reshape(8, 4)
    g = [float(mpmath.e ** (-_mp(cfg["eta_ang"]) * (mpmath.mpf(r) - _mp(m)) ** 2)) for m in cfg["ang_shift"]]
    np.testing.assert_allclose(ang[:, 1], 2.0 * fc * np.array(g), rtol=1e-10)
    np.testing.assert_allclose(ang.reshape(-1), [float(t) for t in terms], rtol=1e-12)


def test_mm_channel_single_charge_closed_form():
    w = sy.model_weights(HCNO_MM, seed=5)
    pos = np.array([[10.0, 10.0, 10.0]])
    Z = np.array([6])
    mm_pos = np.array([[13.0, 11.0, 9.5]])
    mm_q = np.array([-0.834])
    x = orc.evaluate(pos, Z, HCNO_MM, w, box=None, mm_pos=mm_pos, mm_q=mm_q, forces=False, return_x=True)["x"]
    r = mpmath.sqrt(mpmath.mpf(9) + 1 + mpmath.mpf("0.25"))
    phi = mpmath.mpf(sy.KE_COULOMB) * mpmath.mpf(-0.834) * mp_fc(r, mpmath.mpf(12)) / r
    assert x.shape == (1, 385)
    assert abs(x[0, -1] - float(phi)) < 1e-13 * abs(float(phi))
    assert np.all(x[0, :-1] == 0.0)


def _constant_output_weights(cfg, e0, q0):
    """Every W and hidden bias zero, output bias (e0, q0): h3 = CELU(0) = 0, so
    e_i = e0 and q_i = q0 for every atom."""
    w = sy.model_weights(cfg, seed=1)
    out = []
    for layers in w[0]:
        new = [(np.zeros_like(W), np.zeros_like(b)) for W, b in layers]
        new[-1] = (new[-1][0], np.array([e0, q0], np.float32))
        out.append(new)
    return [out]


def test_charge_head_single_charge_closed_form():
    """Predicted charge q in the MM potential: E = e0 + q0 phi with
    phi = ke Q fc(r; 12)/r; the force on the ML atom is q0 ke Q f'(r) u (u the
    unit vector to the MM atom, f = fc/r) and the MM atom feels the opposite."""
    e0, q0 = 0.25, -0.375
    w = _constant_output_weights(HCNO_EE, e0, q0)
    pos = np.array([[10.0, 10.0, 10.0]])
    Z = np.array([6])
    mm_pos = np.array([[13.0, 11.0, 9.5]])
    Q = -0.834
    ref = orc.evaluate(pos, Z, HCNO_EE, w, box=None, mm_pos=mm_pos, mm_q=np.array([Q]))
    d = [mpmath.mpf(3), mpmath.mpf(1), mpmath.mpf("-0.5")]
    r = mpmath.sqrt(sum(a * a for a in d))
    R = mpmath.mpf(12)
    ke = mpmath.mpf(sy.KE_COULOMB)
    fc = mp_fc(r, R)
    E = _mp(np.float32(e0)) + _mp(np.float32(q0)) * ke * _mp(Q) * fc / r
    dfc = -mpmath.pi / (2 * R) * mpmath.sin(mpmath.pi * r / R)
    fprime = (dfc * r - fc) / (r * r)
    F = [_mp(np.float32(q0)) * ke * _mp(Q) * fprime * a / r for a in d]
    assert abs(ref["E"] - float(E)) < 1e-13 * abs(float(E))
    for k in range(3):
        assert abs(ref["F"][0, k] - float(F[k])) < 1e-12 * max(1.0, abs(float(F[k])))
        assert abs(ref["F_mm"][0, k] + float(F[k])) < 1e-12 * max(1.0, abs(float(F[k])))


def test_charge_head_reduces_to_energy_only_model():
    """With the charge row of the output layer zero the two-output model is the
    one-output model with the same other weights."""
    sys_ = sy.solute_in_water(seed=0, n_solute=12, n_side=8, L=24.8, n_keep=300)
    w_ee = sy.model_weights(HCNO_EE, seed=3)
    w_mm = [[[*layers[:-1], (layers[-1][0][:1].copy(), layers[-1][1][:1].copy())] for layers in mem]
            for mem in w_ee]
    for mem in w_ee:
        for layers in mem:
            layers[-1][0][1] = 0.0
            layers[-1][1][1] = 0.0
    args = dict(box=sys_["box"], mm_pos=sys_["mm_pos"], mm_q=sys_["mm_q"])
    a = orc.evaluate(sys_["pos"], sys_["Z"], HCNO_EE, w_ee, **args)
    b = orc.evaluate(sys_["pos"], sys_["Z"], HCNO_MM, w_mm, **args)
    assert abs(a["E"] - b["E"]) < 1e-12 * abs(b["E"])
    np.testing.assert_allclose(a["F"], b["F"], rtol=0, atol=1e-12)
    np.testing.assert_allclose(a["F_mm"], b["F_mm"], rtol=0, atol=1e-12)


def test_charge_head_forces_fd():
    """Central differences of E for NNP and MM atoms with the charge head (the
    q_i phi_i term couples both networks' outputs and the MM geometry)."""
    sys_ = sy.solute_in_water(seed=0, n_solute=12, n_side=8, L=24.8, n_keep=300)
    w = sy.model_weights(HCNO_EE, seed=3)
    args = dict(box=sys_["box"], mm_pos=sys_["mm_pos"].astype(np.float64), mm_q=sys_["mm_q"])
    pos = sys_["pos"].astype(np.float64)
    ref = orc.evaluate(pos, sys_["Z"], HCNO_EE, w, **args)
    assert np.abs(ref["F"].sum(0) + ref["F_mm"].sum(0)).max() < 1e-10
    h = 1e-4
    for a in (0, 7):
        for k in range(3):
            p1 = pos.copy(); p1[a, k] += h
            p2 = pos.copy(); p2[a, k] -= h
            fd = -(orc.evaluate(p1, sys_["Z"], HCNO_EE, w, forces=False, **args)["E"]
                   - orc.evaluate(p2, sys_["Z"], HCNO_EE, w, forces=False, **args)["E"]) / (2 * h)
            assert abs(fd - ref["F"][a, k]) < 2e-7 * max(1.0, abs(ref["F"][a, k]))
    j = int(np.argmax(np.abs(ref["F_mm"]).sum(1)))
    for k in range(3):
        m1 = args["mm_pos"].copy(); m1[j, k] += h
        m2 = args["mm_pos"].copy(); m2[j, k] -= h
        e1 = orc.evaluate(pos, sys_["Z"], HCNO_EE, w, forces=False, **{**args, "mm_pos": m1})["E"]
        e2 = orc.evaluate(pos, sys_["Z"], HCNO_EE, w, forces=False, **{**args, "mm_pos": m2})["E"]
        assert abs(-(e1 - e2) / (2 * h) - ref["F_mm"][j, k]) < 2e-7 * max(1.0, abs(ref["F_mm"][j, k]))


# ------------------------------------------------------------- library routines
def test_celu_matches_torch():
    u = torch.linspace(-3, 3, 2001, dtype=torch.float64)
    np.testing.assert_allclose(orc.celu(u, 0.1).numpy(), torch.nn.functional.celu(u, alpha=0.1).numpy(),
                               rtol=1e-15, atol=1e-17)


def test_cutoff_values():
    r = torch.tensor([0.0, 2.6, 5.2, 6.0], dtype=torch.float64)
    np.testing.assert_allclose(orc.cutoff(r, 5.2).numpy(), [1.0, 0.5, 0.0, 0.0], atol=1e-15)


def test_mlp_matches_torch_nn(w_hcno):
    rng = np.random.default_rng(3)
    x = rng.normal(size=(40, 384))
    sig = rng.integers(0, 4, size=40)
    e = orc.mlp_energies(torch.tensor(x), sig, w_hcno[0], 0.1).numpy()
    ref = np.zeros(40)
    for s in range(4):
        layers = []
        for l, (W, b) in enumerate(w_hcno[0][s]):
            lin = torch.nn.Linear(W.shape[1], W.shape[0]).double()
            with torch.no_grad():
                lin.weight.copy_(torch.tensor(W.astype(np.float64)))
                lin.bias.copy_(torch.tensor(b.astype(np.float64)))
            layers.append(lin)
            if l < 3:
                layers.append(torch.nn.CELU(alpha=0.1))
        net = torch.nn.Sequential(*layers)
        rows = sig == s
        with torch.no_grad():
            ref[rows] = net(torch.tensor(x[rows])).numpy()[:, 0]
    np.testing.assert_allclose(e, ref, rtol=1e-13, atol=1e-13)


def test_pair_class_order():
    P = orc.pair_class_table(4)
    names = "HCNO"
    order = sorted(((P[a, b], names[a] + names[b]) for a in range(4) for b in range(a, 4)))
    assert [n for _, n in order] == ["HH", "HC", "HN", "HO", "CC", "CN", "CO", "NN", "NO", "OO"]


# ------------------------------------------------------------------ neighbours
def test_kdtree_pairs_equal_bruteforce(box64):
    pos, Z, box = box64
    a = orc.neighbour_pairs(pos, 5.2, box)
    b = orc.neighbour_pairs_bruteforce(pos, 5.2, box)
    assert np.array_equal(a[0], b[0]) and np.array_equal(a[1], b[1])
    rng = np.random.Generator(np.random.PCG64(7))
    p, z = sy.walk_molecule(120, rng)
    a = orc.neighbour_pairs(p, 3.5, None)
    b = orc.neighbour_pairs_bruteforce(p, 3.5, None)
    assert np.array_equal(a[0], b[0]) and np.array_equal(a[1], b[1])


def test_neighbour_counts_match_water_density(box64):
    pos, Z, box = box64
    I, J = orc.neighbour_pairs(pos, 5.2, box)
    # 0.1003 atoms / A^3 within a 5.2 A sphere -> ~59 neighbours per atom
    assert 50 < I.size / pos.shape[0] < 68


# ------------------------------------------------------------------ invariants
def _signed_perm(k):
    perms = [(0, 1, 2), (1, 2, 0), (2, 0, 1), (0, 2, 1), (2, 1, 0), (1, 0, 2)]
    p = perms[k % 6]
    s = np.array([1 if (k >> b) & 1 == 0 else -1 for b in range(3)])
    M = np.zeros((3, 3))
    for r, c in enumerate(p):
        M[r, c] = s[r]
    return M


def test_periodic_invariances(box64, w_water):
    pos, Z, box = box64
    pos = pos.astype(np.float64)
    ref = orc.evaluate(pos, Z, WATER, w_water, box=box)
    # zero net force (translation invariance)
    assert np.abs(ref["F"].sum(0)).max() < 1e-11
    # translation
    t = np.array([3.3, -7.1, 11.9])
    r2 = orc.evaluate(pos + t, Z, WATER, w_water, box=box)
    assert abs(r2["E"] - ref["E"]) < 1e-11 * abs(ref["E"])
    np.testing.assert_allclose(r2["F"], ref["F"], atol=1e-11)
    # signed axis permutations of the cube (a subset of the 48, incl. reflections)
    for k in (1, 5, 10, 19, 36, 47):
        M = _signed_perm(k)
        rk = orc.evaluate(pos @ M.T, Z, WATER, w_water, box=box)
        assert abs(rk["E"] - ref["E"]) < 1e-11 * abs(ref["E"]), k
        np.testing.assert_allclose(rk["F"], ref["F"] @ M.T, atol=1e-11)
    # permutation of same-element atoms
    rng = np.random.default_rng(0)
    perm = np.arange(len(Z))
    for z in (1, 8):
        sel = np.nonzero(Z == z)[0]
        perm[sel] = sel[rng.permutation(sel.size)]
    rp = orc.evaluate(pos[perm], Z[perm], WATER, w_water, box=box)
    assert abs(rp["E"] - ref["E"]) < 1e-11 * abs(ref["E"])
    np.testing.assert_allclose(rp["F"], ref["F"][perm], atol=1e-11)


def test_nonperiodic_rotation_and_torque(w_hcno):
    rng = np.random.Generator(np.random.PCG64(11))
    pos, Z = sy.walk_molecule(60, rng)
    pos = pos.astype(np.float64)
    ref = orc.evaluate(pos, Z, HCNO, w_hcno)
    assert np.abs(ref["F"].sum(0)).max() < 1e-11
    c = pos.mean(0)
    tau = np.cross(pos - c, ref["F"]).sum(0)
    assert np.abs(tau).max() < 1e-10
    q, _ = np.linalg.qr(np.random.default_rng(2).normal(size=(3, 3)))
    if np.linalg.det(q) < 0:
        q[:, 0] *= -1
    rr = orc.evaluate((pos - c) @ q.T + c, Z, HCNO, w_hcno)
    assert abs(rr["E"] - ref["E"]) < 1e-11 * abs(ref["E"])
    np.testing.assert_allclose(rr["F"], ref["F"] @ q.T, atol=1e-10)


def test_forces_match_central_differences(box64, w_water):
    pos, Z, box = box64
    pos = pos.astype(np.float64)
    ref = orc.evaluate(pos, Z, WATER, w_water, box=box)
    rng = np.random.default_rng(3)
    h = 1e-4
    for a in rng.choice(len(Z), 5, replace=False):
        for k in range(3):
            p1 = pos.copy()
            p1[a, k] += h
            p2 = pos.copy()
            p2[a, k] -= h
            e1 = orc.evaluate(p1, Z, WATER, w_water, box=box, forces=False)["E"]
            e2 = orc.evaluate(p2, Z, WATER, w_water, box=box, forces=False)["E"]
            fd = -(e1 - e2) / (2 * h)
            assert abs(fd - ref["F"][a, k]) < 2e-7 * max(1.0, abs(ref["F"][a, k])), (a, k)


def test_forces_fd_hcno_and_mm():
    sys_ = sy.solute_in_water(seed=0, n_solute=12, n_side=8, L=24.8, n_keep=300)
    w = sy.model_weights(HCNO_MM, seed=3)
    args = dict(box=sys_["box"], mm_pos=sys_["mm_pos"].astype(np.float64), mm_q=sys_["mm_q"])
    pos = sys_["pos"].astype(np.float64)
    ref = orc.evaluate(pos, sys_["Z"], HCNO_MM, w, **args)
    # Newton's third law across the ML / MM split
    tot = ref["F"].sum(0) + ref["F_mm"].sum(0)
    assert np.abs(tot).max() < 1e-10
    h = 1e-4
    for a in (0, 5):
        for k in range(3):
            p1 = pos.copy(); p1[a, k] += h
            p2 = pos.copy(); p2[a, k] -= h
            fd = -(orc.evaluate(p1, sys_["Z"], HCNO_MM, w, forces=False, **args)["E"]
                   - orc.evaluate(p2, sys_["Z"], HCNO_MM, w, forces=False, **args)["E"]) / (2 * h)
            assert abs(fd - ref["F"][a, k]) < 2e-7 * max(1.0, abs(ref["F"][a, k]))
    # one MM atom
    j = int(np.argmax(np.abs(ref["F_mm"]).sum(1)))
    for k in range(3):
        m1 = args["mm_pos"].copy(); m1[j, k] += h
        m2 = args["mm_pos"].copy(); m2[j, k] -= h
        e1 = orc.evaluate(pos, sys_["Z"], HCNO_MM, w, forces=False, **{**args, "mm_pos": m1})["E"]
        e2 = orc.evaluate(pos, sys_["Z"], HCNO_MM, w, forces=False, **{**args, "mm_pos": m2})["E"]
        assert abs(-(e1 - e2) / (2 * h) - ref["F_mm"][j, k]) < 2e-7 * max(1.0, abs(ref["F_mm"][j, k]))


def test_energy_continuous_across_cutoffs(w_water):
    # radial cutoff: an O-H dimer crossing 5.2 A; angular: a third atom crossing
    # 3.5 A from the O.  A jump in E or in F at the crossing would show up in the
    # second difference across it; smooth E gives O(delta^2).
    for rc, base in ((5.2, np.array([[0.0, 0, 0], [0.0, 0, 0]])),
                     (3.5, np.array([[0.0, 0, 0], [1.0, 0.3, 0], [0.0, 0, 0]]))):
        Z = np.array([8, 1]) if base.shape[0] == 2 else np.array([8, 1, 1])
        direction = np.array([0.3, 0.8, -0.52])
        direction /= np.linalg.norm(direction)
        Es, Fs = [], []
        delta = 1e-6
        for r in (rc - delta, rc, rc + delta):
            p = base.copy()
            p[-1] = r * direction
            res = orc.evaluate(p, Z, WATER, w_water)
            Es.append(res["E"])
            Fs.append(res["F"])
        assert abs(Es[0] - 2 * Es[1] + Es[2]) < 1e-10
        assert np.abs(Fs[0] - Fs[2]).max() < 1e-5


def test_chunking_and_centre_subsets(box64, w_water):
    pos, Z, box = box64
    full = orc.evaluate(pos, Z, WATER, w_water, box=box)
    ch = orc.evaluate(pos, Z, WATER, w_water, box=box, chunk=17)
    assert abs(full["E"] - ch["E"]) < 1e-11 * abs(full["E"])
    np.testing.assert_allclose(ch["F"], full["F"], atol=1e-12)
    # exact forces on one atom from the atoms whose energies depend on it
    a = 37
    I, J = orc.neighbour_pairs(pos, 5.2, box, centres=[a])
    cs = np.unique(np.concatenate([[a], J]))
    sub = orc.evaluate(pos, Z, WATER, w_water, box=box, centres=cs)
    np.testing.assert_allclose(sub["F"][a], full["F"][a], atol=1e-12)
    np.testing.assert_allclose(sub["e"], full["e"][cs], rtol=1e-13)


def test_index_group_subset(box64, w_water):
    pos, Z, box = box64
    idx = np.arange(0, 96)  # first 32 waters form the NNP group
    r = orc.evaluate(pos, Z, WATER, w_water, box=box, nnp_idx=idx)
    ref = orc.evaluate(pos[idx], Z[idx], WATER, w_water, box=box)
    assert abs(r["E"] - ref["E"]) < 1e-12 * abs(ref["E"])
    assert np.all(r["F"][96:] == 0)
    np.testing.assert_allclose(r["F"][idx], ref["F"], atol=1e-13)


def test_ensemble_is_member_mean(box64):
    pos, Z, box = box64
    w8 = sy.model_weights(WATER, seed=1, n_members=3)
    r = orc.evaluate(pos, Z, WATER, w8, box=box)
    parts = [orc.evaluate(pos, Z, WATER, [m], box=box) for m in w8]
    assert abs(r["E"] - np.mean([p["E"] for p in parts])) < 1e-11 * abs(r["E"])
    np.testing.assert_allclose(r["F"], np.mean([p["F"] for p in parts], axis=0), atol=1e-12)


def test_unknown_species_rejected(w_water):
    with pytest.raises(ValueError):
        orc.evaluate(np.zeros((2, 3)), np.array([8, 6]), WATER, w_water)


# --------------------------------------------------------- integer definitions
def test_cell_list_definition(box64):
    pos, Z, box = box64
    sig = orc.species_index(Z, WATER["species"])
    cl = orc.cell_list_fp32(pos, sig, 2, box, WATER["rc_rad"])
    n = len(Z)
    perm, key = cl["perm"], cl["key"]
    assert np.array_equal(np.sort(perm), np.arange(n))
    ks = key[perm]
    assert np.all(np.diff(ks) >= 0)
    same = np.diff(ks) == 0
    assert np.all(np.diff(perm)[same] > 0)          # stable: atom order kept inside a bin
    assert np.array_equal(np.diff(cl["bin_start"]), np.bincount(key, minlength=cl["bin_start"].size - 1))
    # every atom's wrapped position lies in its cell (float64 check with slack)
    nc = cl["n_c"]
    L = box.astype(np.float64)
    w = pos.astype(np.float64) % L
    c = np.stack([(cl["cell"] // (nc[1] * nc[2])), (cl["cell"] // nc[2]) % nc[1], cl["cell"] % nc[2]], 1)
    lo = c * L / nc
    hi = (c + 1) * L / nc
    assert np.all(w >= lo - 1e-4) and np.all(w <= hi + 1e-4)
    assert list(nc) == [2, 2, 2]


def test_fp32_predicate_agrees_with_fp64_away_from_cutoff(box64):
    pos, Z, box = box64
    a = set(zip(*orc.neighbours_fp32(pos, WATER["rc_rad"], box)))
    b = set(zip(*orc.neighbour_pairs_bruteforce(pos, float(WATER["rc_rad"]), box)))
    diff = a ^ b
    p = pos.astype(np.float64)
    for i, j in diff:
        d = p[j] - p[i]
        d -= box * np.rint(d / box)
        assert abs(np.linalg.norm(d) - float(WATER["rc_rad"])) < 1e-4


# -------------------------------------------------------------- generators
def test_water_generator_geometry():
    pos, Z, box = sy.water_box(64, 12.42, seed=0)
    p = pos.astype(np.float64).reshape(-1, 3, 3)
    d1 = np.linalg.norm(p[:, 1] - p[:, 0], axis=1)
    d2 = np.linalg.norm(p[:, 2] - p[:, 0], axis=1)
    assert np.allclose(d1, 0.9572, atol=2e-6) and np.allclose(d2, 0.9572, atol=2e-6)
    cosang = np.sum((p[:, 1] - p[:, 0]) * (p[:, 2] - p[:, 0]), 1) / (d1 * d2)
    assert np.allclose(np.degrees(np.arccos(cosang)), 104.52, atol=2e-4)
    # density 1.0 g/cm^3 within 0.1 %
    mass = 64 * 18.015 / 6.02214076e23
    vol = (12.42e-8) ** 3
    assert abs(mass / vol - 1.0) < 1e-3
    assert list(np.bincount(Z)[[1, 8]]) == [128, 64]


def test_walk_generator_constraints():
    pos, Z, off = sy.walk_batch(8, seed=4)
    sizes = np.diff(off)
    assert np.all((sizes >= 24) & (sizes <= 300))
    for m in range(8):
        p = pos[off[m]:off[m + 1]].astype(np.float64)
        assert np.all(p >= 0) and np.all(p < 40)
        d = np.linalg.norm(p[:, None] - p[None], axis=-1) + np.eye(len(p)) * 10
        assert d.min() >= 0.9 - 1e-5
        for a in range(1, len(p)):
            assert d[a, :a].min() <= 1.5 + 1e-5       # bonded to an earlier atom
    assert set(np.unique(Z)) <= {1, 6, 7, 8}


def test_weight_statistics():
    w = sy.model_weights(HCNO, seed=1)
    W, b = w[0][0][0]
    assert W.shape == (256, 384) and W.dtype == np.float32
    std = math.sqrt(2.0 / (384 + 256))
    assert abs(W.std() / std - 1) < 0.02 and abs(W.mean()) < 0.01 * std * 10
    assert abs(b.std() / 0.1 - 1) < 0.2
    # deterministic and seed dependent
    assert np.array_equal(sy.model_weights(HCNO, seed=1)[0][3][2][0], w[0][3][2][0])
    assert not np.array_equal(sy.model_weights(HCNO, seed=2)[0][0][0][0], W)


def test_splitmix64_published_vector():
    # first outputs of SplitMix64 seeded with 1234567 (Vigna's reference implementation)
    out = sy.splitmix64(1234567, np.arange(5, dtype=np.uint64))
    assert [int(v) for v in out] == [6457827717110365317, 3203168211198807973, 9817491932198370423,
                                     4593380528125082431, 16408922859458223821]


def test_maxwell_boltzmann_temperature():
    pos, Z, box = sy.water_box(64, 12.42, seed=0)
    v = sy.maxwell_boltzmann(Z, 300.0, seed=2)
    m = np.array([sy.WATER_MASS[int(z)] for z in Z])
    assert np.abs((m[:, None] * v).sum(0)).max() < 1e-12
    ke = 0.5 * np.sum(m[:, None] * v * v) / sy.ACC_UNIT
    T = 2 * ke / ((3 * len(Z) - 3) * sy.KB_EV)
    assert abs(T - 300.0) < 1e-9


def test_link_atom_geometry():
    r_ml = np.array([[1.0, 2.0, 3.0]])
    r_mm = np.array([[2.2, 1.1, 4.5]])
    rl = orc.link_atom_positions(r_ml, r_mm, 1.0).numpy()
    assert abs(np.linalg.norm(rl - r_ml) - 1.0) < 1e-14
    u = (r_mm - r_ml) / np.linalg.norm(r_mm - r_ml)
    assert np.allclose(np.cross(rl - r_ml, u), 0, atol=1e-15)


def test_link_atom_defaults_fixture():
    import os
    path = os.path.join(os.path.dirname(__file__), "golden", "link_atom_defaults.txt")
    vals = {}
    for line in open(path):
        if line.strip() and not line.startswith("#"):
            k, v = line.split()
            vals[k] = float(v)
    assert vals["link_atom_atomic_number"] == 1
    d = vals["link_atom_distance_angstrom"]
    # the oracle's default distance is the paper's default
    import inspect
    assert inspect.signature(orc.link_atom_positions).parameters["d"].default == d
    r_ml = np.array([[0.0, 0.0, 0.0]])
    r_mm = np.array([[1.53, 0.0, 0.0]])   # a C-C bond cut by the index group
    rl = orc.link_atom_positions(r_ml, r_mm).numpy()
    np.testing.assert_allclose(rl, [[1.0, 0.0, 0.0]], atol=1e-15)


def test_link_atoms_chain_rule_fd(w_hcno):
    """Link atoms (eq. 4): forces on the ML and MM atoms of a cut bond match
    central differences of the energy, and the link force is redistributed
    without loss (translation invariance of the ML subsystem plus links)."""
    rng = np.random.Generator(np.random.PCG64(21))
    pos, Z = sy.walk_molecule(30, rng)
    pos = pos.astype(np.float64)
    idx = np.arange(18)                          # the index group cuts the chain
    d = np.linalg.norm(pos[:, None] - pos[None], axis=-1)
    ml, mmi = [], []
    for a in idx:
        for b in range(18, 30):
            if d[a, b] < 1.6:
                ml.append(a)
                mmi.append(b)
    assert ml, "test geometry has no cut bond"
    links = (np.array(ml), np.array(mmi), 1.0, 1)
    ref = orc.evaluate(pos, Z, HCNO, w_hcno, nnp_idx=idx, links=links)
    assert np.abs(ref["F"].sum(0)).max() < 1e-10
    touched = sorted(set(idx) | set(mmi))
    untouched = [a for a in range(30) if a not in touched]
    assert np.all(ref["F"][untouched] == 0.0)
    h = 1e-4
    for a in (ml[0], mmi[0], idx[3]):
        for k in range(3):
            p1 = pos.copy(); p1[a, k] += h
            p2 = pos.copy(); p2[a, k] -= h
            fd = -(orc.evaluate(p1, Z, HCNO, w_hcno, nnp_idx=idx, links=links, forces=False)["E"]
                   - orc.evaluate(p2, Z, HCNO, w_hcno, nnp_idx=idx, links=links, forces=False)["E"]) / (2 * h)
            assert abs(fd - ref["F"][a, k]) < 2e-7 * max(1.0, abs(ref["F"][a, k])), (a, k)


# ------------------------------------------------- mechanical embedding (eq. 3)
def _lj_coul_mp(r, qi, qj, si, sj, ei, ej, ke):
    """Coulomb + 12-6 Lennard-Jones of one pair in 30-digit mpmath, Lorentz-Berthelot mixing."""
    r = mpmath.mpf(r)
    s = (mpmath.mpf(si) + mpmath.mpf(sj)) / 2
    e = mpmath.sqrt(mpmath.mpf(ei) * mpmath.mpf(ej))
    return mpmath.mpf(ke) * mpmath.mpf(qi) * mpmath.mpf(qj) / r + 4 * e * ((s / r) ** 12 - (s / r) ** 6)


def test_me_coupling_dimer_closed_form():
    pi = np.array([[0.41, 3.1, 0.0065]])
    pj = np.array([[-0.834, 3.15, 0.0066]])
    xi = np.array([[1.0, 2.0, 3.0]])
    u = np.array([0.48, -0.6, 0.64])          # unit vector
    r = 3.7
    yj = xi + r * u
    E, Fml, Fmm = orc.me_coupling(xi, pi, yj, pj, sy.KE_COULOMB)
    args = (0.41, -0.834, 3.1, 3.15, 0.0065, 0.0066, sy.KE_COULOMB)
    ref = _lj_coul_mp(r, *args)
    dEdr = mpmath.diff(lambda t: _lj_coul_mp(t, *args), r)
    assert abs(E - float(ref)) < 1e-13 * abs(float(ref))
    np.testing.assert_allclose(Fmm[0], -float(dEdr) * u, rtol=1e-11, atol=1e-14)
    np.testing.assert_allclose(Fml[0], float(dEdr) * u, rtol=1e-11, atol=1e-14)


def test_me_coupling_lj_minimum():
    """Neutral pair at r = 2^(1/6) sigma_ij: E = -eps_ij and no force."""
    pi = np.array([[0.0, 2.9, 0.004]])
    pj = np.array([[0.0, 3.3, 0.009]])
    s, e = 3.1, math.sqrt(0.004 * 0.009)
    r = 2.0 ** (1.0 / 6.0) * s
    E, Fml, Fmm = orc.me_coupling(np.zeros((1, 3)), pi, np.array([[0.0, 0.0, r]]), pj, sy.KE_COULOMB)
    assert abs(E + e) < 1e-15
    assert np.abs(Fmm).max() < 1e-12 and np.abs(Fml).max() < 1e-12


def test_me_coupling_cutoff_and_minimum_image():
    """One MM atom inside the cutoff across the periodic boundary, one outside: the
    energy is the closed-form dimer energy at the wrapped distance of the first."""
    L = np.array([20.0, 20.0, 20.0])
    pi = np.array([[0.3, 3.0, 0.005]])
    pj = np.array([[-0.4, 3.2, 0.007], [0.9, 3.4, 0.008]])
    xi = np.array([[0.5, 10.0, 10.0]])
    yj = np.array([[19.0, 10.0, 10.0],       # 1.5 A away through the x boundary
                   [0.5, 10.0, 18.0]])       # 8 A away, beyond the 6 A cutoff
    E, _, Fmm = orc.me_coupling(xi, pi, yj, pj, sy.KE_COULOMB, box=L, cutoff=6.0)
    ref = _lj_coul_mp(1.5, 0.3, -0.4, 3.0, 3.2, 0.005, 0.007, sy.KE_COULOMB)
    assert abs(E - float(ref)) < 1e-12 * abs(float(ref))
    assert np.all(Fmm[1] == 0.0)


def test_me_coupling_third_law_and_fd():
    rng = np.random.default_rng(5)
    L = np.array([18.0, 18.0, 18.0])
    ml = rng.uniform(6, 12, (7, 3))
    mm = rng.uniform(0, 18, (40, 3))
    pml = np.column_stack([rng.uniform(-0.5, 0.5, 7), rng.uniform(2.5, 3.8, 7), rng.uniform(0.001, 0.01, 7)])
    pmm = np.column_stack([rng.uniform(-0.8, 0.8, 40), rng.uniform(2.5, 3.8, 40), rng.uniform(0.001, 0.01, 40)])
    E, Fml, Fmm = orc.me_coupling(ml, pml, mm, pmm, sy.KE_COULOMB, box=L, cutoff=8.5)
    tot = Fml.sum(0) + Fmm.sum(0)
    assert np.abs(tot).max() < 1e-10 * np.abs(Fmm).max()
    h = 1e-5
    for arr, F, idx in ((ml, Fml, 3), (mm, Fmm, 11)):
        for k in range(3):
            p, m = arr.copy(), arr.copy()
            p[idx, k] += h
            m[idx, k] -= h
            args_p = (p, pml, mm, pmm) if arr is ml else (ml, pml, p, pmm)
            args_m = (m, pml, mm, pmm) if arr is ml else (ml, pml, m, pmm)
            Ep = orc.me_coupling(*args_p, sy.KE_COULOMB, box=L, cutoff=8.5, forces=False)[0]
            Em = orc.me_coupling(*args_m, sy.KE_COULOMB, box=L, cutoff=8.5, forces=False)[0]
            fd = -(Ep - Em) / (2 * h)
            assert abs(fd - F[idx, k]) < 1e-6 * max(1.0, abs(F[idx, k]))


# ------------------------------------------- link atoms across a periodic boundary
def _images_nearest(r_ml, r_mm, L):
    """Brute force: the periodic copy r_mm + L k (k in {-4..4}^3) nearest to r_ml."""
    ks = np.array([(a, b, c) for a in range(-4, 5) for b in range(-4, 5) for c in range(-4, 5)], np.float64)
    cands = r_mm[None, :] + ks * L[None, :]
    return cands[np.argmin(np.linalg.norm(cands - r_ml[None, :], axis=1))]


def test_link_atom_minimum_image_brute_force():
    """With a box, the link atom lies on the bond to the nearest periodic copy of the
    MM atom, whatever image the caller's coordinates hold (nearest copy found by
    enumerating images, not by rounding)."""
    rng = np.random.default_rng(11)
    L = np.array([21.0, 23.5, 19.25])
    for _ in range(50):
        r_ml = rng.uniform(0, 1, 3) * L
        bond = rng.normal(size=3)
        bond *= rng.uniform(1.0, 1.6) / np.linalg.norm(bond)
        r_mm = r_ml + bond + L * rng.integers(-3, 4, size=3)       # any image
        near = _images_nearest(r_ml, r_mm, L)
        expect = r_ml + 1.0 * (near - r_ml) / np.linalg.norm(near - r_ml)
        got = orc.link_atom_positions(r_ml[None], r_mm[None], 1.0, box=L).numpy()[0]
        np.testing.assert_allclose(got, expect, atol=1e-12)
        assert abs(np.linalg.norm(got - r_ml) - 1.0) < 1e-12


def _cut_chain(pos, idx, n_all, cutoff=1.6):
    d = np.linalg.norm(pos[:, None] - pos[None], axis=-1)
    ml, mm = [], []
    for a in idx:
        for b in range(n_all):
            if b not in set(idx) and d[a, b] < cutoff:
                ml.append(a)
                mm.append(b)
    return np.array(ml), np.array(mm)


def test_link_atoms_periodic_boundary_translation(w_hcno):
    """A periodic ML subsystem with link atoms: translating every atom so that a cut
    bond straddles the box face, then wrapping each atom into [0, L), leaves E and
    every force unchanged.  (A link placed along the raw, unwrapped bond vector
    would land about one box length away and change E.)"""
    rng = np.random.Generator(np.random.PCG64(21))
    pos, Z = sy.walk_molecule(30, rng)
    pos = pos.astype(np.float64)
    L = np.array([44.0, 44.0, 44.0])
    idx = np.arange(18)
    ml, mm = _cut_chain(pos, idx, 30)
    assert ml.size
    links = (ml, mm, 1.0, 1)
    ref = orc.evaluate(pos, Z, HCNO, w_hcno, box=L, nnp_idx=idx, links=links)
    # put the first cut bond's midpoint on the x = 0 face, then wrap every atom
    mid = 0.5 * (pos[ml[0]] + pos[mm[0]])
    shift = np.array([-mid[0], 3.7 - mid[1], 5.1 - mid[2]])
    moved = pos + shift
    wrapped = moved - L * np.floor(moved / L)
    assert abs(wrapped[ml[0], 0] - wrapped[mm[0], 0]) > L[0] / 2, "the cut bond must straddle the face"
    got = orc.evaluate(wrapped, Z, HCNO, w_hcno, box=L, nnp_idx=idx, links=links)
    assert abs(got["E"] - ref["E"]) < 1e-10 * max(1.0, abs(ref["E"]))
    np.testing.assert_allclose(got["F"], ref["F"], atol=1e-9)


def test_link_atoms_straddling_bond_fd(w_hcno):
    """Central differences of E on the ML and MM atoms of a cut bond that crosses
    the periodic boundary (wrapped coordinates) match the oracle's forces."""
    rng = np.random.Generator(np.random.PCG64(21))
    pos, Z = sy.walk_molecule(30, rng)
    pos = pos.astype(np.float64)
    L = np.array([44.0, 44.0, 44.0])
    idx = np.arange(18)
    ml, mm = _cut_chain(pos, idx, 30)
    mid = 0.5 * (pos[ml[0]] + pos[mm[0]])
    moved = pos + np.array([-mid[0], 0.0, 0.0])
    pos = moved - L * np.floor(moved / L)
    links = (ml, mm, 1.0, 1)
    ref = orc.evaluate(pos, Z, HCNO, w_hcno, box=L, nnp_idx=idx, links=links)
    h = 1e-4
    for a in (ml[0], mm[0]):
        for k in range(3):
            p1 = pos.copy(); p1[a, k] += h
            p2 = pos.copy(); p2[a, k] -= h
            e1 = orc.evaluate(p1, Z, HCNO, w_hcno, box=L, nnp_idx=idx, links=links, forces=False)["E"]
            e2 = orc.evaluate(p2, Z, HCNO, w_hcno, box=L, nnp_idx=idx, links=links, forces=False)["E"]
            fd = -(e1 - e2) / (2 * h)
            assert abs(fd - ref["F"][a, k]) < 2e-7 * max(1.0, abs(ref["F"][a, k])), (a, k, fd, ref["F"][a, k])


# ---------------------------------------------------------- network input gradient
def test_mlp_input_grad_central_differences(w_water, w_hcno):
    """d e_i / d x_i of ``mlp_input_grad`` against central differences of the atomic
    energies in float64, for random descriptor rows of both networks."""
    rng = np.random.default_rng(8)
    for cfg, w in ((WATER, w_water[0]), (HCNO, w_hcno[0])):
        D = cfg["widths"][0]
        S = len(cfg["species"])
        x = rng.uniform(0.0, 1.5, size=(2 * S, D))
        sig = np.arange(2 * S) % S
        e, g = orc.mlp_input_grad(x, sig, w, cfg["celu_alpha"])
        h = 1e-5
        cols = rng.choice(D, 12, replace=False)
        for r in range(x.shape[0]):
            for c in cols:
                xp = x.copy(); xp[r, c] += h
                xm = x.copy(); xm[r, c] -= h
                ep = orc.mlp_energies(torch.tensor(xp), sig, w, cfg["celu_alpha"]).numpy()[r]
                em = orc.mlp_energies(torch.tensor(xm), sig, w, cfg["celu_alpha"]).numpy()[r]
                fd = (ep - em) / (2 * h)
                assert abs(fd - g[r, c]) < 1e-7 * max(1.0, abs(g[r, c])), (r, c, fd, g[r, c])


def test_mlp_input_grad_linear_regime_closed_form():
    """With every hidden pre-activation positive, CELU is the identity and the network
    is the affine map W4 W3 W2 W1 x + const, so d e / d x = (W4 W3 W2 W1)[0]: a
    product of the weight matrices by numpy matmul, independent of the autograd path."""
    rng = np.random.default_rng(2)
    widths = [128, 160, 128, 96, 1]
    layers = []
    for l in range(4):
        W = np.abs(rng.normal(0, 0.05, size=(widths[l + 1], widths[l])))   # non-negative
        b = np.full(widths[l + 1], 0.5)
        layers.append((W, b))
    x = rng.uniform(0.0, 1.0, size=(3, 128))                                 # non-negative inputs
    e, g = orc.mlp_input_grad(x, np.zeros(3, np.int64), [layers], 0.1)
    J = layers[3][0] @ layers[2][0] @ layers[1][0] @ layers[0][0]
    np.testing.assert_allclose(g, np.repeat(J, 3, axis=0), rtol=1e-12, atol=1e-14)
    h = x
    for W, b in layers:
        h = h @ W.T + b
    np.testing.assert_allclose(e, h[:, 0], rtol=1e-12)


# ------------------------------------------------- k-d tree FP32 neighbour oracle
@pytest.mark.parametrize("case", ["c1", "shifted", "open"])
def test_kdtree_fp32_pairs_equal_bruteforce(case):
    """``neighbours_fp32_kdtree`` (used for boxes too large for the O(N^2) scan) returns
    exactly the pair set of the brute-force float32 definition, for both cutoffs."""
    if case == "c1":
        pos, Z, box = sy.water_box(64, 12.42, seed=0)
    elif case == "shifted":
        pos, Z, box = sy.water_box(1000, 31.07, seed=5)
        k = np.random.default_rng(3).integers(-3, 4, size=pos.shape)
        pos = (pos + k * np.asarray(box)).astype(np.float32)
    else:
        pos, Z, _ = sy.walk_batch(6, seed=2)
        box = None
    for rc in (5.2, 3.5):
        I, J = orc.neighbours_fp32(pos, rc, box)
        I2, J2 = orc.neighbours_fp32_kdtree(pos, rc, box)
        assert np.array_equal(I, I2) and np.array_equal(J, J2)


def test_kdtree_fp32_pairs_equal_bruteforce_12288():
    """The same equality on the 4,096-water (12,288-atom) box at the radial cutoff."""
    pos, Z, box = sy.water_box(4096, 49.7, seed=0)
    I, J = orc.neighbours_fp32(pos, 5.2, box)
    I2, J2 = orc.neighbours_fp32_kdtree(pos, 5.2, box)
    assert I.size > 700000
    assert np.array_equal(I, I2) and np.array_equal(J, J2)


def test_periodic_batch_equals_separate_systems(w_water):
    """evaluate_batch with per-system boxes: each system as its own periodic call; a
    zero box row is an open system."""
    a = sy.water_box(64, 12.42, seed=0)
    b = sy.water_box(80, 13.38, seed=1)
    pos = np.concatenate([a[0], b[0]])
    Z = np.concatenate([a[1], b[1]])
    off = np.array([0, 192, 432])
    boxes = np.array([a[2], [0.0, 0.0, 0.0]], np.float32)
    E, F = orc.evaluate_batch(pos, Z, off, WATER, w_water, boxes=boxes)
    ra = orc.evaluate(a[0], a[1], WATER, w_water, box=a[2])
    rb = orc.evaluate(b[0], b[1], WATER, w_water, box=None)
    assert E[0] == ra["E"] and E[1] == rb["E"]
    np.testing.assert_array_equal(F[:192], ra["F"])
    np.testing.assert_array_equal(F[192:], rb["F"])
