"""GPU parity: the HIP path through the C ABI against the FP64 oracle.

Integer stages (cell binning, the stable counting sort, neighbour sets) are
compared bit for bit with the oracle's FP32 definitions; floating-point stages
within the stated tolerances:
  FP32 form: force relative RMSE <= 1e-5, energy error per atom <= 1e-6 eV;
  BF16 form: force relative RMSE <= 1e-2.
"""
import math

import numpy as np
import pytest
import torch

import oracle as orc
import synthetic as sy

pytestmark = pytest.mark.gpu

WATER = sy.model_config("water")
HCNO = sy.model_config("hcno")
HCNO_MM = sy.model_config("hcno_mm")
HCNO_EE = sy.model_config("hcno_ee")


def _lib():
    if not torch.cuda.is_available():
        pytest.fail("GPU test run without a visible GPU")
    import paper_2604_21441_amd as P
    return P


def rel_rmse(F, Fref):
    return float(np.linalg.norm(F - Fref) / np.linalg.norm(Fref))


def worst_atom(F, Fref):
    """Largest per-atom force error relative to the RMS atomic force of the reference: a
    few badly wrong atoms cannot hide in a norm over many atoms (BF16 rounding gives a few
    times the relative RMSE; one wrong atom is of order 1)."""
    err = np.linalg.norm(F - Fref, axis=1)
    return float(err.max() / np.sqrt(np.mean(np.sum(Fref ** 2, axis=1))))


BF16_ATOM_BOUND = 0.15


@pytest.fixture(scope="module")
def P():
    return _lib()


@pytest.fixture(scope="module")
def w_water():
    return sy.model_weights(WATER, seed=1)


@pytest.fixture(scope="module")
def w_hcno():
    return sy.model_weights(HCNO, seed=1)


@pytest.fixture(scope="module")
def water_models(P, w_water):
    flat = sy.flat_weights(w_water)
    return {p: P.NNPModel(WATER, weights=flat, precision=p) for p in ("fp32", "bf16")}


@pytest.fixture(scope="module")
def boxes():
    # "large" (18,432 atoms, 10^3 cells x 2 species): a second periodic size on the
    # fused one-chunk scan-and-scatter path; the multi-chunk scan (more than 16,384
    # bins) is checked bit for bit in test_gpu_full_size.py
    c2 = sy.water_box(4096, 49.7, seed=0)
    # "c2s": the same box with every atom moved by whole box lengths (-3..3 per
    # component), so that positions lie far outside [0, L)
    k = np.random.default_rng(3).integers(-3, 4, size=c2[0].shape)
    c2s = ((c2[0] + k * np.asarray(c2[2])).astype(c2[0].dtype), c2[1], c2[2])
    return {"c1": sy.water_box(64, 12.42, seed=0), "c2": c2, "c2s": c2s,
            "large": sy.water_box(6144, 56.9, seed=0)}


@pytest.fixture(scope="module")
def oracle_res(boxes, w_water):
    out = {}
    for k, (pos, Z, box) in boxes.items():
        if k != "large":
            out[k] = orc.evaluate(pos, Z, WATER, w_water, box=box, return_x=True)
    return out


def _run(model, pos, Z, box, **kw):
    d = torch.from_numpy(pos).cuda()
    E, F, Fmm = model.compute(d, Z, box, **kw)
    torch.cuda.synchronize()
    assert model.status() == 0
    return E.cpu().numpy(), F.cpu().numpy(), (None if Fmm is None else Fmm.cpu().numpy())


# ------------------------------------------------------------ integer stages
@pytest.mark.parametrize("name", ["c1", "c2", "large"])
def test_cell_list_bit_exact(P, water_models, boxes, name):
    pos, Z, box = boxes[name]
    m = water_models["fp32"]
    _run(m, pos, Z, box)
    sigma = orc.species_index(Z, WATER["species"])
    ref = orc.cell_list_fp32(pos, sigma, 2, box, WATER["rc_rad"])
    grid = m.read(P._lib.NNP_BUF_GRID)
    assert list(grid[1:]) == list(ref["n_c"])
    assert np.array_equal(m.read(P._lib.NNP_BUF_KEY), ref["key"])
    assert np.array_equal(m.read(P._lib.NNP_BUF_PERM), ref["perm"])
    assert np.array_equal(m.read(P._lib.NNP_BUF_BIN_START), ref["bin_start"])
    # visiting order: bin by bin, species by species, ascending slot
    bs, nb = ref["bin_start"], len(ref["bin_start"]) // 2
    expect = np.concatenate([np.arange(bs[s * nb + b], bs[s * nb + b + 1]) for b in range(nb) for s in range(2)])
    assert np.array_equal(m.read(P._lib.NNP_BUF_ORDER), expect)


@pytest.mark.parametrize("name", ["c1", "c2", "c2s", "large"])
def test_neighbour_sets_bit_exact(P, water_models, boxes, name):
    pos, Z, box = boxes[name]
    m = water_models["fp32"]
    _run(m, pos, Z, box)
    perm = m.read(P._lib.NNP_BUF_PERM)
    cnt = m.read(P._lib.NNP_BUF_NBR_COUNT)
    sigma = orc.species_index(Z, WATER["species"])
    for buf, rc, col in ((P._lib.NNP_BUF_NBR_RAD, WATER["rc_rad"], 0), (P._lib.NNP_BUF_NBR_ANG, WATER["rc_ang"], 1)):
        lists = m.read(buf)
        I, J = orc.neighbours_fp32(pos, rc, box)
        ref = set(zip(I.tolist(), J.tolist()))
        got = set()
        for i in range(len(perm)):
            row = lists[i, :cnt[i, col]]
            sp = sigma[perm[row]]
            assert np.all(np.diff(sp) >= 0), "neighbour row not grouped by species"
            got.update((int(perm[i]), int(perm[j])) for j in row)
        assert got == ref


# ------------------------------------------------------- floating-point stages
@pytest.mark.parametrize("name", ["c1", "c2"])
def test_descriptors_fp32(P, water_models, boxes, oracle_res, name):
    pos, Z, box = boxes[name]
    m = water_models["fp32"]
    _run(m, pos, Z, box)
    perm = m.read(P._lib.NNP_BUF_PERM)
    x = m.read(P._lib.NNP_BUF_DESCRIPTOR)[:, :128]
    xr = np.empty_like(x, dtype=np.float64)
    xr[perm] = x
    ref = oracle_res[name]["x"]
    err = np.linalg.norm(xr - ref, axis=1) / np.linalg.norm(ref, axis=1)
    # FP32 with hardware exp2/log2: the angular power (1 + cos)^zeta is exp2(zeta log2(.)),
    # which multiplies log2's absolute error (~1e-7) by zeta = 14.1, so a row can carry a
    # few 1e-6 of relative error; 5e-6 bounds that with margin.
    assert err.max() < 5e-6, err.max()


@pytest.mark.parametrize("name", ["c1", "c2"])
def test_network_stage_fp32(P, water_models, boxes, oracle_res, w_water, name):
    pos, Z, box = boxes[name]
    m = water_models["fp32"]
    _run(m, pos, Z, box)
    perm = m.read(P._lib.NNP_BUF_PERM)
    e = np.empty(len(perm))
    e[perm] = m.read(P._lib.NNP_BUF_ATOM_ENERGY)
    g = m.read(P._lib.NNP_BUF_DEDX)[:, :128]
    gr = np.empty(g.shape)
    gr[perm] = g
    sigma = orc.species_index(Z, WATER["species"])
    e_ref, g_ref = orc.mlp_input_grad(oracle_res[name]["x"], sigma, w_water[0], WATER["celu_alpha"])
    assert np.abs(e - e_ref).max() < 2e-5 * max(1.0, np.abs(e_ref).max())
    assert rel_rmse(gr, g_ref) < 1e-5


@pytest.mark.parametrize("name", ["c1", "c2"])
def test_energy_forces_fp32(P, water_models, boxes, oracle_res, name):
    pos, Z, box = boxes[name]
    E, F, _ = _run(water_models["fp32"], pos, Z, box)
    ref = oracle_res[name]
    n = len(Z)
    assert abs(E[0] - ref["E"]) / n < 1e-6
    assert rel_rmse(F, ref["F"]) < 1e-5
    assert np.abs(F.sum(0)).max() < 1e-6 * np.abs(F).max() * math.sqrt(n)


@pytest.mark.parametrize("name", ["c1", "c2"])
def test_energy_forces_bf16(P, water_models, boxes, oracle_res, name):
    pos, Z, box = boxes[name]
    E, F, _ = _run(water_models["bf16"], pos, Z, box)
    ref = oracle_res[name]
    n = len(Z)
    assert abs(E[0] - ref["E"]) / n < 2e-3
    assert rel_rmse(F, ref["F"]) < 1e-2
    assert worst_atom(F, ref["F"]) < BF16_ATOM_BOUND


def test_forces_match_gpu_finite_differences(P, water_models, boxes):
    """The adjoint agrees with central differences of the GPU's own FP32 energy."""
    pos, Z, box = boxes["c2"]
    m = water_models["fp32"]
    E0, F, _ = _run(m, pos, Z, box)
    rng = np.random.default_rng(3)
    h = 3e-3
    for a in rng.choice(len(Z), 32, replace=False):
        for k in range(3):
            p1 = pos.copy(); p1[a, k] += h
            p2 = pos.copy(); p2[a, k] -= h
            dh = float(p1[a, k]) - float(p2[a, k])
            e1 = _run(m, p1, Z, box)[0][0]
            e2 = _run(m, p2, Z, box)[0][0]
            fd = -(e1 - e2) / dh
            assert abs(fd - F[a, k]) < 3e-3 * max(1.0, abs(F[a, k])), (a, k, fd, F[a, k])


def test_index_group_subset(P, water_models, boxes, w_water):
    pos, Z, box = boxes["c1"]
    rng = np.random.default_rng(5)
    idx = np.sort(rng.choice(len(Z), 100, replace=False)).astype(np.int32)
    E, F, _ = _run(water_models["fp32"], pos, Z, box, nnp_idx=idx)
    ref = orc.evaluate(pos, Z, WATER, w_water, box=box, nnp_idx=idx)
    assert abs(E[0] - ref["E"]) / idx.size < 1e-6
    mask = np.ones(len(Z), bool)
    mask[idx] = False
    assert np.all(F[mask] == 0.0)
    assert rel_rmse(F[idx], ref["F"][idx]) < 1e-5


def test_accumulate_and_determinism(P, water_models, boxes):
    pos, Z, box = boxes["c2"]
    m = water_models["fp32"]
    d = torch.from_numpy(pos).cuda()
    E1, F1, _ = m.compute(d, Z, box)
    E2, F2, _ = m.compute(d, Z, box)
    torch.cuda.synchronize()
    assert E1.item() == E2.item()                       # fixed-order FP64 energy sum
    assert torch.allclose(F1, F2, rtol=0, atol=1e-10)   # FP64 atomics: order only
    m.compute(d, Z, box, accumulate_into=(E1, F1, None))
    torch.cuda.synchronize()
    assert abs(E1.item() - 2 * E2.item()) < 1e-9 * abs(E2.item())
    assert torch.allclose(F1, 2 * F2, rtol=1e-12, atol=1e-10)


def test_autograd_function(P, water_models, boxes):
    pos, Z, box = boxes["c1"]
    m = water_models["fp32"]
    x = torch.from_numpy(pos).cuda().requires_grad_(True)
    E = m.energy(x, Z, box)
    E.backward()
    _, F, _ = m.compute(x.detach(), Z, box)
    assert torch.allclose(x.grad.double(), -F.double(), rtol=1e-5, atol=1e-6)


def test_graph_replay_matches_eager(P, water_models, boxes):
    """Replays of the captured call equal direct launches, with eager work and syncs between replays."""
    pos, Z, box = boxes["c2"]
    m = water_models["fp32"]
    d = torch.from_numpy(pos).cuda()
    m.set_graph(False)
    E0, F0, _ = m.compute(d, Z, box)
    torch.cuda.synchronize()
    E0, F0 = E0.clone(), F0.clone()
    m.set_graph(True)
    E = torch.empty(1, dtype=torch.float64, device="cuda")
    F = torch.empty((len(Z), 3), dtype=torch.float64, device="cuda")
    for rep in range(4):
        E.fill_(123.0)
        F.fill_(-7.0)
        m.compute(d, Z if rep == 0 else None, box, out=(E, F, None))
        torch.cuda.synchronize()
        junk = torch.randn(1000, device="cuda").sum()   # unrelated eager work between replays
        torch.cuda.synchronize()
        assert abs(E.item() - E0.item()) < 1e-12 * abs(E0.item()), rep
        assert torch.allclose(F, F0, rtol=0, atol=1e-12), rep
    # a different size is a different configuration: captured anew, not replayed
    pos_s, Z_s, box_s = boxes["c1"]
    Es, Fs, _ = m.compute(torch.from_numpy(pos_s).cuda(), Z_s, box_s)
    m.set_graph(False)
    Es2, Fs2, _ = m.compute(torch.from_numpy(pos_s).cuda(), Z_s, box_s)
    m.set_graph(True)
    torch.cuda.synchronize()
    assert abs(Es.item() - Es2.item()) < 1e-12 * abs(Es2.item())
    assert torch.allclose(Fs, Fs2, rtol=0, atol=1e-12)
    m.compute(d, Z, box, out=(E, F, None))
    torch.cuda.synchronize()
    assert abs(E.item() - E0.item()) < 1e-12 * abs(E0.item())
    # a moved configuration through the same graph gives the new answer
    d2 = d + 0.01
    torch.cuda.synchronize()
    d.copy_(d2)
    m.compute(d, None, box, out=(E, F, None))
    m.set_graph(False)
    E2, F2, _ = m.compute(d, None, box)
    torch.cuda.synchronize()
    assert abs(E.item() - E2.item()) < 1e-12 * abs(E2.item())
    m.set_graph(True)


def test_autotune_keeps_results(P, w_water):
    """Every kernel variant the autotuner may pick computes the same energy and forces."""
    pos, Z, box = sy.water_box(4096, 49.7, seed=0)
    d = torch.from_numpy(pos).cuda()
    for prec in ("fp32", "bf16"):
        m = P.NNPModel(WATER, weights=sy.flat_weights(w_water), precision=prec)
        E0, F0, _ = m.compute(d, Z, box)
        torch.cuda.synchronize()
        E0, F0 = E0.clone(), F0.clone()
        chosen = m.autotune(3)
        assert 0 <= chosen["network"] < 10 and chosen["neighbours"] in (0, 1, 2, 3)
        assert chosen["descriptor"] in (0, 1, 2, 3, 4) and chosen["adjoint"] in (0, 1, 2)
        E1, F1, _ = m.compute(d, Z, box)
        torch.cuda.synchronize()
        assert m.status() == 0
        # Variants differ only in summation order.  In the BF16 form a descriptor
        # value that differs in its last FP32 bit can round to the neighbouring
        # BF16 network input (2^-8 relative), a few of the 1.6M inputs per call:
        # force differences of a few 1e-5 (against 7e-3 for BF16 vs the oracle).
        e_tol, f_tol = (1e-6, 1e-5) if prec == "fp32" else (1e-5, 2e-4)
        assert abs(E1.item() - E0.item()) / len(Z) < e_tol
        assert rel_rmse(F1.cpu().numpy(), F0.cpu().numpy()) < f_tol
        m.close()


VARIANTS = [("neighbours", 0, "fp32"), ("neighbours", 1, "fp32"), ("neighbours", 2, "fp32"),
            ("neighbours", 3, "fp32"), ("descriptor", 0, "fp32"), ("descriptor", 2, "fp32"),
            ("descriptor", 1, "fp32"), ("descriptor", 3, "fp32"), ("descriptor", 4, "fp32"), ("network", 0, "fp32"), ("network", 1, "fp32"), ("network", 2, "fp32"),
            ("network", 3, "fp32"), ("network", 4, "fp32"), ("network", 5, "fp32"), ("network", 6, "fp32"),
            ("network", 7, "fp32"), ("network", 0, "bf16"), ("network", 1, "bf16"), ("network", 2, "bf16"),
            ("network", 3, "bf16"), ("network", 4, "bf16"), ("network", 5, "bf16"), ("network", 6, "bf16"),
            ("network", 7, "bf16"), ("network", 8, "bf16"), ("network", 9, "bf16"), ("network", 8, "fp32"), ("adjoint", 0, "fp32"),
            ("adjoint", 1, "fp32"), ("adjoint", 2, "fp32")]


@pytest.mark.parametrize("stage,variant,prec", VARIANTS)
def test_pinned_variant_parity(P, w_water, boxes, oracle_res, stage, variant, prec):
    """Each kernel variant, pinned through the C ABI, against the oracle (c2, 12,288 atoms)."""
    pos, Z, box = boxes["c2"]
    m = P.NNPModel(WATER, weights=sy.flat_weights(w_water), precision=prec)
    m.set_variant(stage, variant)
    E, F, _ = _run(m, pos, Z, box)
    ref = oracle_res["c2"]
    n = len(Z)
    if prec == "fp32":
        assert abs(E[0] - ref["E"]) / n < 1e-6
        assert rel_rmse(F, ref["F"]) < 1e-5
    else:
        assert abs(E[0] - ref["E"]) / n < 2e-3
        assert rel_rmse(F, ref["F"]) < 1e-2
        assert worst_atom(F, ref["F"]) < BF16_ATOM_BOUND
    perm = m.read(P._lib.NNP_BUF_PERM)
    x = m.read(P._lib.NNP_BUF_DESCRIPTOR)[:, :128]
    xr = np.empty(x.shape)
    xr[perm] = x
    err = np.linalg.norm(xr - ref["x"], axis=1) / np.linalg.norm(ref["x"], axis=1)
    assert err.max() < 1e-5, err.max()
    nvar = {"network": 10, "neighbours": 4, "descriptor": 5, "adjoint": 3}[stage]
    for bad in ((stage, nvar), (4, 0), (stage, -2)):
        with pytest.raises(P.NNPError) as ex:
            m.set_variant(*bad)
        assert ex.value.status == P._lib.NNP_EINVAL
    m.set_variant(stage, -1)
    m.close()


def test_mixed_network_tiling_bit_identical(P, w_water, w_hcno, boxes):
    """The mixed tiling (16-atom tiles for the species with the fewest atoms)
    changes only which workgroup computes an atom: every atom's network output
    and hence every force is bit-identical to the uniform 32-atom tiling, and
    the energy differs at most by the FP64 summation order of the partials."""
    pos, Z, box = boxes["c2"]
    out = {}
    for v in (2, 4):
        m = P.NNPModel(WATER, weights=sy.flat_weights(w_water), precision="fp32")
        m.set_variant("network", v)
        out[v] = _run(m, pos, Z, box)
        assert m.variants()["network"] == v
        m.close()
    assert np.array_equal(out[2][1], out[4][1])
    assert abs(out[2][0][0] - out[4][0][0]) <= 1e-12 * abs(out[2][0][0])
    # batched open systems (per-system energies summed from the atomic ones)
    pos, Z, off = sy.walk_batch(12, seed=5)
    d = torch.from_numpy(pos).cuda()
    res = {}
    for v in (2, 4):
        m = P.NNPModel(HCNO, weights=sy.flat_weights(w_hcno), precision="bf16")
        m.set_variant("network", v)
        E, F = m.compute_batch(d, Z, off)
        torch.cuda.synchronize()
        assert m.status() == 0
        res[v] = (E.cpu().numpy(), F.cpu().numpy())
        m.close()
    assert np.array_equal(res[2][0], res[4][0])
    assert np.array_equal(res[2][1], res[4][1])


@pytest.mark.parametrize("prec", ["fp32", "bf16"])
def test_network_variants_bitwise_forces(P, w_water, boxes, prec):
    """All network kernels 0-7 run the same matrix-core sequence per atom (same K
    order, same operand rounding: BF16 activations are rounded once, by the
    layer that produces them), so dE/dx and hence every force is bitwise the
    same whichever kernel ran.  (Variant 8 takes celu' from the BF16-rounded
    activation; it is compared with a tolerance in test_lds_network_kernel.)"""
    pos, Z, box = boxes["c2"]
    ref = None
    for v in range(8):
        m = P.NNPModel(WATER, weights=sy.flat_weights(w_water), precision=prec)
        m.set_variant("network", v)
        F = _run(m, pos, Z, box)[1]
        m.close()
        if ref is None:
            ref = F
        assert np.array_equal(F, ref), f"network variant {v}"


def test_lds_network_kernel(P, w_water, boxes, oracle_res):
    """Network variants 8 and 9 (BF16 weights resident in LDS, one 32- or 16-atom tile per
    wavefront, transposed LDS reads for the backward products) against the oracle like every
    BF16 kernel, and against variant 2 within BF16 rounding: the CELU is one fma and a
    median and the output-layer dot product is summed in another order (FP32 rounding,
    which can move a BF16-rounded activation by one BF16 ulp), and celu' comes from
    min(exp(u / alpha), 1) kept in FP16 for the hidden layers (relative 2^-10), where
    variant 2 computes it in FP32 from the FP32 activation."""
    for name in ("c1", "c2"):
        pos, Z, box = boxes[name]
        out = {}
        for v in (2, 8, 9):
            m = P.NNPModel(WATER, weights=sy.flat_weights(w_water), precision="bf16")
            m.set_variant("network", v)
            E, F, _ = _run(m, pos, Z, box)
            e = m.read(P._lib.NNP_BUF_ATOM_ENERGY).copy()
            g = m.read(P._lib.NNP_BUF_DEDX).copy()
            assert m.variants()["network"] == v
            out[v] = (E, F, e, g)
            m.close()
        ref = oracle_res[name]
        for v in (8, 9):
            # the CELU is evaluated as one fma (alpha t - alpha) instead of a subtraction
            # and a product; an activation whose FP32 value moves by one ulp can round to
            # the neighbouring BF16 value (2^-8 relative), so atomic energies agree to
            # BF16 input rounding, not bitwise
            de = np.abs(out[v][2] - out[2][2])
            assert de.max() < 5e-4, (name, v, de.max())                      # atomic energies
            assert abs(out[v][0][0] - out[2][0][0]) / len(Z) < 1e-5, (name, v)
            # celu' differs by at most 2^-10 relative per element (FP16 derivative);
            # three backward layers: a few 1e-3 relative
            assert rel_rmse(out[v][3], out[2][3]) < 5e-3, (name, v)          # dE/dx
            assert rel_rmse(out[v][1], out[2][1]) < 5e-3, (name, v)          # forces
            e2, ev = rel_rmse(out[2][1], ref["F"]), rel_rmse(out[v][1], ref["F"])
            print(f"{name}: force rel RMSE vs oracle, BF16 variant 2 {e2:.3e}, variant {v} {ev:.3e}")
            assert ev < 1e-2 and worst_atom(out[v][1], ref["F"]) < BF16_ATOM_BOUND
        # the two LDS tilings do the same arithmetic per atom
        assert np.array_equal(out[8][1], out[9][1]), name
    # an FP32 model pinned to variant 8 runs the default kernel instead
    m = P.NNPModel(WATER, weights=sy.flat_weights(w_water), precision="fp32")
    m.set_variant("network", 8)
    _run(m, *boxes["c1"])
    assert m.variants()["network"] == 2
    m.close()


def test_adjoint_wide_reverse_search_bit_identical(P, w_water, w_hcno, boxes):
    """Adjoint variant 2 finds each centre's place in its neighbours' lists by
    counting with wide loads instead of a binary search; the places, hence
    every force, are the same bit for bit.  Covered: water boxes of two sizes,
    open H/C/N/O molecules (uneven species segments), and a radial capacity
    that is not a multiple of four (rows not 16-byte aligned: the variant
    falls back to the binary search)."""
    cases = [("c1", None), ("c2", None), ("c2", 126)]
    for name, cap in cases:
        pos, Z, box = boxes[name]
        F = {}
        for v in (0, 2):
            m = P.NNPModel(WATER, weights=sy.flat_weights(w_water))
            if cap is not None:
                m.reserve(len(Z), max_rad_nbr=cap)
            m.set_variant("adjoint", v)
            F[v] = _run(m, pos, Z, box)[1]
            m.close()
        assert np.array_equal(F[0], F[2]), (name, cap)
    pos, Z, off = sy.walk_batch(24, seed=9)
    d = torch.from_numpy(pos).cuda()
    F = {}
    for v in (0, 2):
        m = P.NNPModel(HCNO, weights=sy.flat_weights(w_hcno))
        m.set_variant("adjoint", v)
        E, Fv = m.compute_batch(d, Z, off)
        torch.cuda.synchronize()
        assert m.status() == 0
        F[v] = Fv.cpu().numpy()
        m.close()
    assert np.array_equal(F[0], F[2])


@pytest.mark.parametrize("prec", ["fp32", "bf16"])
def test_network_variants_bitwise_forces_wide(P, w_hcno, prec):
    """The same bitwise agreement for the wide H/C/N/O networks: the batched
    walk molecules (384 inputs) and the solute with the MM channel (416 after
    padding), including the MM forces."""
    pos, Z, off = sy.walk_batch(24, seed=9)
    d = torch.from_numpy(pos).cuda()
    ref = None
    for v in range(8):
        m = P.NNPModel(HCNO, weights=sy.flat_weights(w_hcno), precision=prec)
        m.set_variant("network", v)
        E, F = m.compute_batch(d, Z, off)
        torch.cuda.synchronize()
        assert m.status() == 0
        F = F.cpu().numpy()
        m.close()
        if ref is None:
            ref = F
        assert np.array_equal(F, ref), f"network variant {v}"
    sysd = sy.solute_in_water(seed=0)
    w = sy.model_weights(HCNO_MM, seed=3)
    mm_pos, mm_q = torch.from_numpy(sysd["mm_pos"]).cuda(), torch.from_numpy(sysd["mm_q"]).cuda()
    ref = None
    for v in range(8):
        m = P.NNPModel(HCNO_MM, weights=sy.flat_weights(w), precision=prec)
        m.set_variant("network", v)
        _, F, Fmm = _run(m, sysd["pos"], sysd["Z"], sysd["box"], mm_pos=mm_pos, mm_q=mm_q)
        m.close()
        if ref is None:
            ref = (F, Fmm)
        # forces on the NNP atoms are bitwise equal; MM forces are FP64 sums in
        # atomic order, so equal to rounding
        assert np.array_equal(F, ref[0]), f"network variant {v}"
        assert np.allclose(Fmm, ref[1], rtol=0, atol=1e-12 * max(1.0, np.abs(ref[1]).max())), f"variant {v}"


def test_neighbour_sets_batched_and_open(P, w_hcno):
    pos, Z, off = sy.walk_batch(6, seed=7)
    m = P.NNPModel(HCNO, weights=sy.flat_weights(w_hcno), precision="fp32")
    m.compute_batch(torch.from_numpy(pos).cuda(), Z, off)
    torch.cuda.synchronize()
    perm = m.read(P._lib.NNP_BUF_PERM)
    sigma = orc.species_index(Z, HCNO["species"])
    sys_of = np.repeat(np.arange(6), np.diff(off))
    key = sigma * 6 + sys_of
    assert np.array_equal(m.read(P._lib.NNP_BUF_KEY), key)
    assert np.array_equal(perm, np.argsort(key, kind="stable"))
    cnt = m.read(P._lib.NNP_BUF_NBR_COUNT)
    lists = m.read(P._lib.NNP_BUF_NBR_RAD)
    ref = set()
    for s in range(6):
        I, J = orc.neighbours_fp32(pos[off[s]:off[s + 1]], HCNO["rc_rad"], None)
        ref.update(zip((I + off[s]).tolist(), (J + off[s]).tolist()))
    got = set()
    for i in range(len(perm)):
        row = lists[i, :cnt[i, 0]]
        assert np.all(np.diff(row) > 0) or np.all(np.diff(sigma[perm[row]]) >= 0)
        got.update((int(perm[i]), int(perm[j])) for j in row)
    assert got == ref
    # one open (non-periodic) system uses the per-atom kernel
    a, b = off[2], off[3]
    m.compute(torch.from_numpy(pos[a:b].copy()).cuda(), Z[a:b], None)
    torch.cuda.synchronize()
    perm = m.read(P._lib.NNP_BUF_PERM)
    cnt = m.read(P._lib.NNP_BUF_NBR_COUNT)
    lists = m.read(P._lib.NNP_BUF_NBR_ANG)
    I, J = orc.neighbours_fp32(pos[a:b], HCNO["rc_ang"], None)
    got = set()
    for i in range(len(perm)):
        got.update((int(perm[i]), int(perm[j])) for j in lists[i, :cnt[i, 1]])
    assert got == set(zip(I.tolist(), J.tolist()))
    m.close()


@pytest.mark.parametrize("n_mem,name", [(3, "c1"), (8, "c1"), (8, "c2")])
def test_ensemble_members_average(P, boxes, n_mem, name):
    """An ensemble of networks sharing one descriptor (the 8-network form is what the
    paper's ANI-2x runs): E and F are the member means, against the oracle's mean over
    members, in both forms and with every network tiling the tuner may pick."""
    pos, Z, box = boxes[name]
    wm = sy.model_weights(WATER, seed=1, n_members=n_mem)
    ref = orc.evaluate(pos, Z, WATER, wm, box=box)
    for prec, tol in (("fp32", 1e-5), ("bf16", 1e-2)):
        for v in ((2, 7) if name == "c2" else (-1,)):
            m = P.NNPModel(WATER, weights=sy.flat_weights(wm), precision=prec, n_members=n_mem)
            if v >= 0:
                m.set_variant("network", v)
            E, F, _ = _run(m, pos, Z, box)
            assert abs(E[0] - ref["E"]) / len(Z) < (1e-6 if prec == "fp32" else 2e-3)
            assert rel_rmse(F, ref["F"]) < tol
            if prec == "bf16":
                assert worst_atom(F, ref["F"]) < BF16_ATOM_BOUND
            m.close()


def test_seeded_weights_match_generator(P):
    """nnp_create's own seed path reproduces the generator module's weights."""
    pos, Z, box = sy.water_box(64, 12.42, seed=0)
    m_seed = P.NNPModel(WATER, seed=7, precision="fp32")
    m_given = P.NNPModel(WATER, weights=sy.flat_weights(sy.model_weights(WATER, seed=7)), precision="fp32")
    E1, F1, _ = _run(m_seed, pos, Z, box)
    E2, F2, _ = _run(m_given, pos, Z, box)
    assert E1[0] == E2[0]
    assert np.array_equal(F1, F2) or np.abs(F1 - F2).max() < 1e-12


def test_nve_energy_error_scales_with_dt_squared(P, water_models):
    """Velocity Verlet with the library's forces: halving dt cuts the energy error ~4x,
    which needs forces consistent with the energy."""
    from paper_2604_21441_amd.md import run_nve
    pos, Z, box = sy.water_box(64, 12.42, seed=0)
    masses = np.array([sy.WATER_MASS[int(z)] for z in Z])
    v0 = sy.maxwell_boltzmann(Z, 300.0, seed=2)
    devs = []
    for dt, steps in ((0.2, 100), (0.1, 200)):
        r = run_nve(water_models["fp32"], pos, Z, box, masses, v0, dt=dt, steps=steps)
        assert np.all(np.isfinite(r["etot"]))
        devs.append(r["max_abs_dev_eV_per_atom"])
    ratio = devs[0] / devs[1]
    assert 2.5 < ratio < 6.0, (devs, ratio)


def test_link_atoms(P, w_hcno):
    """Link atoms on bonds cut by the index group (eq. 4): energy and the forces on
    ML, MM and interior atoms against the oracle's chain rule."""
    rng = np.random.Generator(np.random.PCG64(21))
    pos, Z = sy.walk_molecule(40, rng)
    idx = np.arange(24, dtype=np.int32)
    d = np.linalg.norm(pos[:, None].astype(np.float64) - pos[None], axis=-1)
    ml, mm = [], []
    for a in idx:
        for b in range(24, 40):
            if d[a, b] < 1.6:
                ml.append(a)
                mm.append(b)
    assert ml
    ml = np.array(ml, np.int32)
    mm = np.array(mm, np.int32)
    m = P.NNPModel(HCNO, weights=sy.flat_weights(w_hcno), precision="fp32")
    m.set_links(ml, mm, 1.0, 1)
    for box in (None, np.full(3, 60.0, np.float32)):
        E, F, _ = _run(m, pos, Z, box, nnp_idx=idx)
        ref = orc.evaluate(pos, Z, HCNO, w_hcno, box=box, nnp_idx=idx, links=(ml, mm, 1.0, 1))
        assert abs(E[0] - ref["E"]) / (idx.size + ml.size) < 1e-6
        assert rel_rmse(F, ref["F"]) < 1e-5
        assert np.abs(F[mm]).max() > 0            # MM atoms of cut bonds feel the link atoms
    m.set_links(np.zeros(0, np.int32), np.zeros(0, np.int32))
    E, F, _ = _run(m, pos, Z, None, nnp_idx=idx)
    ref = orc.evaluate(pos, Z, HCNO, w_hcno, nnp_idx=idx)
    assert abs(E[0] - ref["E"]) / idx.size < 1e-6
    assert rel_rmse(F, ref["F"]) < 1e-5
    m.close()


@pytest.mark.parametrize("variant", [0, 1, 2, 3, 4])
def test_descriptor_variants_hcno_batch(P, w_hcno, variant):
    """Each descriptor kernel on an uneven batch of H/C/N/O molecules (ten species-pair
    classes with few pairs each): descriptor rows, molecule energies and forces against the
    oracle, and two calls bitwise equal (the pool kernels add chunk sums with LDS atomics)."""
    pos, Z, off = sy.walk_batch(24, seed=7)
    m = P.NNPModel(HCNO, weights=sy.flat_weights(w_hcno), precision="fp32")
    m.set_variant("descriptor", variant)
    d = torch.from_numpy(pos).cuda()
    xs = []
    for _ in range(2):
        E, F = m.compute_batch(d, Z, off)
        torch.cuda.synchronize()
        assert m.status() == 0
        xs.append(m.read(P._lib.NNP_BUF_DESCRIPTOR)[:, :384].copy())
    assert np.array_equal(xs[0], xs[1])
    E, F = E.cpu().numpy(), F.cpu().numpy()
    perm = m.read(P._lib.NNP_BUF_PERM)
    xr = np.empty(xs[0].shape)
    xr[perm] = xs[0]
    for s in range(len(off) - 1):
        a, b = off[s], off[s + 1]
        ref = orc.evaluate(pos[a:b], Z[a:b], HCNO, w_hcno, return_x=True)
        err = np.linalg.norm(xr[a:b] - ref["x"], axis=1) / np.linalg.norm(ref["x"], axis=1)
        assert err.max() < 5e-6, (s, err.max())
        assert abs(E[s] - ref["E"]) / (b - a) < 1e-6
        assert rel_rmse(F[a:b], ref["F"]) < 1e-5
    m.close()


@pytest.mark.parametrize("variant", [3, 4])
def test_pool_descriptor_dense_and_isolated(P, w_hcno, variant):
    """The pool kernels on a dense H/C/N/O cluster (about 35 angular neighbours per atom, so
    the wavefront's neighbour geometry takes a second pass) plus an isolated atom (every
    unit empty: its row must be zero): descriptor rows, energy and forces against the oracle."""
    rng = np.random.default_rng(11)
    n = 300
    pos = rng.uniform(0.0, 6.0, size=(n, 3))
    keep = [0]
    for k in range(1, n):   # at least 1 A apart: 92 atoms, up to 57 angular neighbours
        if np.min(np.linalg.norm(pos[keep] - pos[k], axis=1)) > 1.0:
            keep.append(k)
    pos = np.concatenate([pos[keep], [[30.0, 30.0, 30.0]]]).astype(np.float32)
    Z = rng.choice(np.array([1, 6, 7, 8], dtype=np.int32), size=len(pos))
    m = P.NNPModel(HCNO, weights=sy.flat_weights(w_hcno), precision="fp32")
    m.set_variant("descriptor", variant)
    E, F, _ = _run(m, pos, Z, None)
    perm = m.read(P._lib.NNP_BUF_PERM)
    x = m.read(P._lib.NNP_BUF_DESCRIPTOR)[:, :384]
    xr = np.empty(x.shape)
    xr[perm] = x
    ref = orc.evaluate(pos, Z, HCNO, w_hcno, return_x=True)
    assert np.all(xr[-1] == 0.0)
    err = np.linalg.norm(xr[:-1] - ref["x"][:-1], axis=1) / np.linalg.norm(ref["x"][:-1], axis=1)
    assert err.max() < 5e-6, err.max()
    assert abs(E[0] - ref["E"]) / len(Z) < 1e-6
    assert rel_rmse(F, ref["F"]) < 1e-5
    # dense enough that two atoms of a wavefront hold more than 64 angular neighbours
    # (the second staging pass)
    d = np.linalg.norm(pos[:-1, None] - pos[None, :-1], axis=2)
    n_ang = (d < HCNO["rc_ang"]).sum(axis=1) - 1
    assert n_ang.mean() > 30 and n_ang.max() < 64
    m.close()


@pytest.fixture(scope="module")
def hcno_periodic(w_hcno):
    """420 H/C/N/O atoms at least 1 A apart (minimum image) in a periodic 14 A box:
    about 27 angular neighbours per atom, pairs across every face."""
    rng = np.random.default_rng(21)
    L = 14.0
    pts = []
    while len(pts) < 420:
        p = rng.uniform(0.0, L, 3)
        if pts:
            d = np.asarray(pts) - p
            d -= L * np.round(d / L)
            if np.min(np.einsum("ij,ij->i", d, d)) < 1.0:
                continue
        pts.append(p)
    pos = np.asarray(pts, dtype=np.float32)
    Z = rng.choice(np.array([1, 6, 7, 8], dtype=np.int32), size=len(pos))
    box = np.array([L, L, L], dtype=np.float32)
    return pos, Z, box, orc.evaluate(pos, Z, HCNO, w_hcno, box=box, return_x=True)


@pytest.mark.parametrize("variant", [1, 3, 4])
def test_descriptor_variants_hcno_periodic(P, w_hcno, hcno_periodic, variant):
    """Row and pool descriptor kernels on a periodic H/C/N/O box (minimum image across the
    faces, ten classes): descriptor rows, energy and forces against the oracle."""
    pos, Z, box, ref = hcno_periodic
    m = P.NNPModel(HCNO, weights=sy.flat_weights(w_hcno), precision="fp32")
    m.set_variant("descriptor", variant)
    E, F, _ = _run(m, pos, Z, box)
    perm = m.read(P._lib.NNP_BUF_PERM)
    x = m.read(P._lib.NNP_BUF_DESCRIPTOR)[:, :384]
    xr = np.empty(x.shape)
    xr[perm] = x
    err = np.linalg.norm(xr - ref["x"], axis=1) / np.linalg.norm(ref["x"], axis=1)
    assert err.max() < 5e-6, err.max()
    assert abs(E[0] - ref["E"]) / len(Z) < 1e-6
    assert rel_rmse(F, ref["F"]) < 1e-5
    m.close()


# ------------------------------------------------------------------ batching
def test_batched_open_systems(P, w_hcno):
    pos, Z, off = sy.walk_batch(12, seed=4)
    flat = sy.flat_weights(w_hcno)
    for prec, tol in (("fp32", 1e-5), ("bf16", 1e-2)):
        m = P.NNPModel(HCNO, weights=flat, precision=prec)
        E, F = m.compute_batch(torch.from_numpy(pos).cuda(), Z, off)
        torch.cuda.synchronize()
        assert m.status() == 0
        E = E.cpu().numpy()
        F = F.cpu().numpy()
        Eref, Fref = orc.evaluate_batch(pos, Z, off, HCNO, w_hcno)
        n = np.diff(off)
        assert np.all(np.abs(E - Eref) / n < (1e-6 if prec == "fp32" else 1e-2))
        assert rel_rmse(F, Fref) < tol
        if prec == "fp32":
            # one batched call equals separate open-system calls
            for s in (0, 5, 11):
                a, b = off[s], off[s + 1]
                Es, Fs, _ = m.compute(torch.from_numpy(pos[a:b].copy()).cuda(), Z[a:b], None)
                torch.cuda.synchronize()
                assert abs(Es.item() - E[s]) < 1e-12 * max(1.0, abs(E[s]))
                assert np.allclose(Fs.cpu().numpy(), F[a:b], rtol=0, atol=1e-9)
        m.close()


# ---------------------------------------------------------------- MM charges
def test_mm_charge_channel(P):
    sysd = sy.solute_in_water(seed=0)
    w = sy.model_weights(HCNO_MM, seed=3)
    ref = orc.evaluate(sysd["pos"], sysd["Z"], HCNO_MM, w, box=sysd["box"], mm_pos=sysd["mm_pos"],
                       mm_q=sysd["mm_q"])
    m = P.NNPModel(HCNO_MM, weights=sy.flat_weights(w), precision="fp32")
    E, F, Fmm = _run(m, sysd["pos"], sysd["Z"], sysd["box"], mm_pos=torch.from_numpy(sysd["mm_pos"]).cuda(),
                     mm_q=torch.from_numpy(sysd["mm_q"]).cuda())
    n = len(sysd["Z"])
    assert abs(E[0] - ref["E"]) / n < 1e-6
    assert rel_rmse(F, ref["F"]) < 1e-5
    Fall = np.concatenate([F, Fmm])
    Fall_ref = np.concatenate([ref["F"], ref["F_mm"]])
    assert rel_rmse(Fall, Fall_ref) < 1e-5
    assert np.abs(F.sum(0) + Fmm.sum(0)).max() < 1e-4


def test_mm_channel_charge_counts(P):
    """The MM channel at the edges of its grid: more charges than 512
    workgroups of 256 lanes cover (each lane then takes several charges), and
    a model with the MM input called with no charges (phi = 0: compared with
    the oracle given zero charges)."""
    sysd = sy.solute_in_water(seed=0)
    w = sy.model_weights(HCNO_MM, seed=3)
    L = float(sysd["box"][0])
    rng = np.random.default_rng(11)
    n_mm = 140_000                                  # > 512 * 256
    y = rng.uniform(0.0, L, size=(2 * n_mm, 3))
    d = y[:, None, :] - sysd["pos"].astype(np.float64)[None, :, :]
    d -= L * np.rint(d / L)
    far = np.min(np.einsum("mak,mak->ma", d, d), axis=1) > 4.0   # no charge within 2 A of the solute
    y = np.ascontiguousarray(y[far][:n_mm].astype(np.float32))
    q = rng.uniform(-0.5, 0.5, size=n_mm)
    q = (q - q.mean()).astype(np.float32)
    ref = orc.evaluate(sysd["pos"], sysd["Z"], HCNO_MM, w, box=sysd["box"], mm_pos=y, mm_q=q)
    m = P.NNPModel(HCNO_MM, weights=sy.flat_weights(w), precision="fp32")
    E, F, Fmm = _run(m, sysd["pos"], sysd["Z"], sysd["box"], mm_pos=torch.from_numpy(y).cuda(),
                     mm_q=torch.from_numpy(q).cuda())
    n = len(sysd["Z"])
    assert abs(E[0] - ref["E"]) / n < 1e-6
    assert rel_rmse(np.concatenate([F, Fmm]), np.concatenate([ref["F"], ref["F_mm"]])) < 1e-5
    # no charges
    zq = np.zeros(4, dtype=np.float32)
    ref0 = orc.evaluate(sysd["pos"], sysd["Z"], HCNO_MM, w, box=sysd["box"], mm_pos=y[:4], mm_q=zq)
    e0 = torch.empty((0, 3), dtype=torch.float32, device="cuda")
    E0, F0, _ = _run(m, sysd["pos"], sysd["Z"], sysd["box"], mm_pos=e0,
                     mm_q=torch.empty((0,), dtype=torch.float32, device="cuda"))
    assert abs(E0[0] - ref0["E"]) / n < 1e-6
    assert rel_rmse(F0, ref0["F"]) < 1e-5
    m.close()


@pytest.mark.parametrize("prec", ["fp32", "bf16"])
def test_predicted_charge_embedding(P, prec):
    """Electrostatic embedding with charges from the network (a second output
    q_i entering as q_i phi_i): energy, NNP and MM forces against the oracle,
    for every network kernel.  Across kernels the forces agree to rounding
    only: q_i is a dot product summed over the wavefronts that own the rows,
    so its FP32 summation order depends on the wavefront count, and q_i
    reaches the forces through dE/dphi_i."""
    sysd = sy.solute_in_water(seed=0)
    w = sy.model_weights(HCNO_EE, seed=3)
    ref = orc.evaluate(sysd["pos"], sysd["Z"], HCNO_EE, w, box=sysd["box"], mm_pos=sysd["mm_pos"],
                       mm_q=sysd["mm_q"])
    mm_pos, mm_q = torch.from_numpy(sysd["mm_pos"]).cuda(), torch.from_numpy(sysd["mm_q"]).cuda()
    n = len(sysd["Z"])
    tol_e, tol_f = (1e-6, 1e-5) if prec == "fp32" else (1e-2, 1e-2)
    x = orc.evaluate(sysd["pos"], sysd["Z"], HCNO_EE, w, box=sysd["box"], mm_pos=sysd["mm_pos"],
                     mm_q=sysd["mm_q"], forces=False, return_x=True)["x"]
    sig = orc.species_index(sysd["Z"], HCNO_EE["species"])
    q_ref = orc.mlp_outputs(torch.tensor(x), sig, w[0], HCNO_EE["celu_alpha"])[:, 1].numpy()
    first = None
    for v in range(8):
        m = P.NNPModel(HCNO_EE, weights=sy.flat_weights(w), precision=prec)
        m.set_variant("network", v)
        E, F, Fmm = _run(m, sysd["pos"], sysd["Z"], sysd["box"], mm_pos=mm_pos, mm_q=mm_q)
        if v == 0:   # the predicted charges themselves, per atom
            qs = np.empty(n)
            qs[m.read(P._lib.NNP_BUF_PERM)] = m.read(P._lib.NNP_BUF_CHARGE)
            np.testing.assert_allclose(qs, q_ref, rtol=0, atol=(1e-5 if prec == "fp32" else 2e-2) * np.abs(q_ref).max())
        m.close()
        assert abs(E[0] - ref["E"]) / n < tol_e, (v, E[0], ref["E"])
        Fall = np.concatenate([F, Fmm])
        assert rel_rmse(Fall, np.concatenate([ref["F"], ref["F_mm"]])) < tol_f, v
        assert np.abs(F.sum(0) + Fmm.sum(0)).max() < 1e-4
        if first is None:
            first = F
        assert rel_rmse(F, first) < 1e-6, f"network variant {v}"


# ------------------------------------------------- caller's pair list (Methods)
def _half_pairs(pos, box, r_list, rng, extra_far=500):
    """Half pair list of every pair closer than r_list (float64), in shuffled order, with
    some far pairs mixed in (the engine's list may reach beyond the cutoff)."""
    I, J = orc.neighbour_pairs(pos, r_list, box)
    keep = I < J
    P = np.stack([I[keep], J[keep]], axis=1)
    far = rng.integers(0, len(pos), size=(extra_far, 2))
    far = far[far[:, 0] < far[:, 1]]
    P = np.unique(np.concatenate([P, far]), axis=0)
    P = P[rng.permutation(len(P))]
    return np.ascontiguousarray(P.astype(np.int32))


def test_pair_list_path_matches_cell_list(P, w_water, boxes):
    """With the engine's pair list (cutoff plus a 0.5 A buffer) the lists, the energy and the
    forces are bit-identical to the cell-list path; also for an index group."""
    rng = np.random.default_rng(11)
    pos, Z, box = boxes["c2"]
    pairs = torch.from_numpy(_half_pairs(pos, box, WATER["rc_rad"] + 0.5, rng)).cuda()
    d = torch.from_numpy(pos).cuda()
    for idx in (None, np.sort(rng.choice(len(Z), 9000, replace=False)).astype(np.int32)):
        a = P.NNPModel(WATER, weights=sy.flat_weights(w_water), precision="fp32")
        b = P.NNPModel(WATER, weights=sy.flat_weights(w_water), precision="fp32")
        Ea, Fa, _ = a.compute(d, Z, box, nnp_idx=idx)
        Eb, Fb, _ = b.compute_pairs(d, pairs, Z, box, nnp_idx=idx)
        torch.cuda.synchronize()
        assert a.status() == 0 and b.status() == 0
        for buf in (P._lib.NNP_BUF_NBR_COUNT, P._lib.NNP_BUF_NBR_RAD, P._lib.NNP_BUF_NBR_ANG, P._lib.NNP_BUF_PERM):
            ra, rb = a.read(buf), b.read(buf)
            if buf in (P._lib.NNP_BUF_NBR_RAD, P._lib.NNP_BUF_NBR_ANG):
                cnt = a.read(P._lib.NNP_BUF_NBR_COUNT)[:, 0 if buf == P._lib.NNP_BUF_NBR_RAD else 1]
                mask = np.arange(ra.shape[1])[None, :] < cnt[:, None]
                ra, rb = np.where(mask, ra, -1), np.where(mask, rb, -1)
            assert np.array_equal(ra, rb), buf
        assert Ea.item() == Eb.item()
        assert torch.equal(Fa, Fb)
        # a second call through the captured graph, with the pair list reused
        Eb2, Fb2, _ = b.compute_pairs(d, pairs, None, box, nnp_idx=idx)
        torch.cuda.synchronize()
        assert Eb2.item() == Ea.item()
        a.close()
        b.close()


def test_pair_list_bad_entries(P, w_water, boxes):
    pos, Z, box = boxes["c1"]
    m = P.NNPModel(WATER, weights=sy.flat_weights(w_water), precision="fp32")
    d = torch.from_numpy(pos).cuda()
    for bad in ([[0, 0]], [[0, len(Z)]], [[3, 7], [3, 7]]):
        pairs = torch.tensor(bad, dtype=torch.int32, device="cuda")
        if bad == [[3, 7], [3, 7]]:
            pos2 = pos.copy()
            pos2[7] = pos2[3] + np.array([1.5, 0.0, 0.0], np.float32)   # make the repeated pair a real one
            d = torch.from_numpy(pos2).cuda()
        m.compute_pairs(d, pairs, Z, box)
        torch.cuda.synchronize()
        assert m.status() == P._lib.NNP_EINVAL, bad
    m.close()


# ------------------------------------------- mechanical embedding (eq. 3)
def test_me_coupling_parity(P):
    """Coulomb + LJ over the 60 x 30,000 ML-MM pairs of the solvated solute, against the oracle:
    periodic with a 12 A cutoff, and open with every pair; then accumulation and error paths."""
    sysd = sy.solute_in_water(seed=0)
    pml = sy.lj_params_solute(sysd["Z"])
    pmm = sy.lj_params_water(len(sysd["mm_q"]) // 3)
    t = lambda a: torch.from_numpy(np.ascontiguousarray(a, np.float32)).cuda()
    xml, qml, xmm, qmm = t(sysd["pos"]), t(pml), t(sysd["mm_pos"]), t(pmm)
    for box, cutoff in ((sysd["box"], 12.0), (None, 0.0)):
        E_ref, Fml_ref, Fmm_ref, Eabs = orc.me_coupling(sysd["pos"], pml, sysd["mm_pos"], pmm, sy.KE_COULOMB,
                                                        box=box, cutoff=cutoff if cutoff > 0 else None,
                                                        return_abs=True)
        E, Fml, Fmm = P.nnp_me_coupling(xml, qml, xmm, qmm, box=box, cutoff=cutoff, ke=sy.KE_COULOMB)
        torch.cuda.synchronize()
        assert abs(E.item() - E_ref) < 1e-6 * Eabs
        F = np.concatenate([Fml.cpu().numpy(), Fmm.cpu().numpy()])
        F_ref = np.concatenate([Fml_ref, Fmm_ref])
        assert rel_rmse(F, F_ref) < 1e-5
        assert np.abs(F.sum(0)).max() < 1e-5 * np.abs(F).max() * math.sqrt(len(F))
    # accumulate: a second call on the same outputs doubles them
    out = P.nnp_me_coupling(xml, qml, xmm, qmm, box=sysd["box"], cutoff=12.0, ke=sy.KE_COULOMB)
    E1, F1 = out[0].item(), out[2].clone()
    P.nnp_me_coupling(xml, qml, xmm, qmm, box=sysd["box"], cutoff=12.0, ke=sy.KE_COULOMB, accumulate=True, out=out)
    torch.cuda.synchronize()
    assert abs(out[0].item() - 2 * E1) < 1e-9 * abs(E1)
    assert torch.allclose(out[2], 2 * F1, rtol=1e-12, atol=0)
    for kw, status in ((dict(box=sysd["box"], cutoff=0.0), P._lib.NNP_EBOX),
                       (dict(box=sysd["box"], cutoff=40.0), P._lib.NNP_EBOX),
                       (dict(box=None, cutoff=-1.0), P._lib.NNP_EINVAL)):
        with pytest.raises(P.NNPError) as ex:
            P.nnp_me_coupling(xml, qml, xmm, qmm, ke=sy.KE_COULOMB, **kw)
        assert ex.value.status == status


# ------------------------------------------------------------- error paths
def test_error_paths(P, w_water):
    m = P.NNPModel(WATER, weights=sy.flat_weights(w_water), precision="fp32")
    pos, Z, box = sy.water_box(64, 12.42, seed=0)
    d = torch.from_numpy(pos).cuda()
    m.reserve(len(Z))
    E = torch.empty(1, dtype=torch.float64, device="cuda")
    F = torch.empty((len(Z), 3), dtype=torch.float64, device="cuda")
    with pytest.raises(P.NNPError) as ex:
        Zb = Z.copy(); Zb[5] = 6
        P.nnp_compute(m.h, d, Zb, box, None, None, None, E, F)
    assert ex.value.status == P._lib.NNP_ESPECIES
    with pytest.raises(P.NNPError) as ex:
        P.nnp_compute(m.h, d, Z, np.array([10.0, 12.42, 12.42], np.float32), None, None, None, E, F)
    assert ex.value.status == P._lib.NNP_EBOX
    big = torch.zeros((len(Z) + 1, 3), dtype=torch.float32, device="cuda")
    with pytest.raises(P.NNPError) as ex:
        P.nnp_compute(m.h, big, np.ones(len(Z) + 1, np.int32), box, None, None, None, E, F)
    assert ex.value.status == P._lib.NNP_ECAPACITY
    # neighbour capacity overflow is reported by the device status word
    m.reserve(len(Z), 1, 0, 4, 2)
    P.nnp_compute(m.h, d, Z, box, None, None, None, E, F)
    assert m.status() == P._lib.NNP_ECAPACITY
    assert m.status() == P._lib.NNP_OK     # cleared by the read
    m.reserve(len(Z))
    bad = pos.copy(); bad[3, 1] = np.nan
    P.nnp_compute(m.h, torch.from_numpy(bad).cuda(), Z, box, None, None, None, E, F)
    assert m.status() == P._lib.NNP_ENONFINITE
    m.close()
