"""GPU parity of the batched, link-atom and graph-update paths through the C ABI.

* Batches of periodic systems with their own boxes (and open systems in the
  same batch) against the oracle's per-system evaluation, and against
  separate single-system calls.
* Link atoms (eq. 4) on a cut bond that crosses the periodic boundary, through
  the cell list and through a caller's pair list (which cannot name link
  atoms), against the oracle's minimum-image placement.
* Graph replay when the box changes every call (a barostat) and when the
  autograd path is called repeatedly: the captured graph is updated or
  replayed, never rebuilt, and the results equal direct launches.
"""
import numpy as np
import pytest
import torch

import oracle as orc
import synthetic as sy

pytestmark = pytest.mark.gpu

WATER = sy.model_config("water")
HCNO = sy.model_config("hcno")


@pytest.fixture(scope="module")
def P():
    if not torch.cuda.is_available():
        pytest.fail("GPU test run without a visible GPU")
    import paper_2604_21441_amd as P
    return P


def rel_rmse(F, Fref):
    return float(np.linalg.norm(F - Fref) / np.linalg.norm(Fref))


def graph_counts(P, m):
    b, u, r = m.read(P._lib.NNP_BUF_GRAPH)
    return int(b), int(u), int(r)


# ------------------------------------------------ batches of periodic boxes
def _water_batch():
    """Three periodic water boxes of different sizes and one open water cluster."""
    parts = [sy.water_box(64, 12.42, seed=0), sy.water_box(80, 13.38, seed=1), sy.water_box(27, 10.9, seed=2),
             sy.water_box(40, 11.0, seed=5)]
    pos = np.concatenate([p[0] for p in parts])
    Z = np.concatenate([p[1] for p in parts])
    off = np.concatenate([[0], np.cumsum([len(p[1]) for p in parts])]).astype(np.int32)
    boxes = np.array([parts[0][2], parts[1][2], parts[2][2], [0.0, 0.0, 0.0]], np.float32)
    return pos, Z, off, boxes


def test_batched_periodic_boxes(P):
    w = sy.model_weights(WATER, seed=1)
    pos, Z, off, boxes = _water_batch()
    Eref, Fref = orc.evaluate_batch(pos, Z, off, WATER, w, boxes=boxes)
    n_at = np.diff(off)
    for prec in ("fp32", "bf16"):
        m = P.NNPModel(WATER, weights=sy.flat_weights(w), precision=prec)
        d = torch.from_numpy(pos).cuda()
        E, F = m.compute_batch(d, Z, off, boxes=boxes)
        torch.cuda.synchronize()
        assert m.status() == 0
        E, F = E.cpu().numpy(), F.cpu().numpy()
        if prec == "fp32":
            assert np.all(np.abs(E - Eref) / n_at < 1e-6), (E, Eref)
            assert rel_rmse(F, Fref) < 1e-5
            # one batched call equals separate single-system calls.  An open system is
            # one bin either way (same lists, same order: equal to FP64 rounding); a
            # single periodic call bins by cells, so its rows list the same neighbours
            # in another order and the FP32 sums differ by rounding only.
            for s in range(len(n_at)):
                a, b = off[s], off[s + 1]
                box = None if not boxes[s].any() else boxes[s]
                Es, Fs, _ = m.compute(torch.from_numpy(pos[a:b].copy()).cuda(), Z[a:b], box)
                torch.cuda.synchronize()
                Fs = Fs.cpu().numpy()
                if box is None:
                    assert abs(Es.item() - E[s]) < 1e-12 * max(1.0, abs(E[s])), s
                    assert np.allclose(Fs, F[a:b], rtol=0, atol=1e-9), s
                else:
                    assert abs(Es.item() - E[s]) / n_at[s] < 1e-7, s
                    assert rel_rmse(Fs, F[a:b]) < 1e-6, s
        else:
            assert np.all(np.abs(E - Eref) / n_at < 2e-3), (E, Eref)
            assert rel_rmse(F, Fref) < 1e-2
        m.close()


@pytest.mark.parametrize("stage,variant", [("descriptor", 0), ("descriptor", 2), ("descriptor", 3),
                                           ("descriptor", 4), ("adjoint", 1), ("adjoint", 2),
                                           ("neighbours", 1)])
def test_batched_periodic_boxes_variants(P, stage, variant):
    """Every kernel variant that reads the per-system boxes, pinned, on the batch of
    periodic boxes and an open cluster: energies and forces against the oracle."""
    w = sy.model_weights(WATER, seed=1)
    pos, Z, off, boxes = _water_batch()
    Eref, Fref = orc.evaluate_batch(pos, Z, off, WATER, w, boxes=boxes)
    m = P.NNPModel(WATER, weights=sy.flat_weights(w), precision="fp32")
    m.set_variant(stage, variant)
    E, F = m.compute_batch(torch.from_numpy(pos).cuda(), Z, off, boxes=boxes)
    torch.cuda.synchronize()
    assert m.status() == 0
    E, F = E.cpu().numpy(), F.cpu().numpy()
    assert np.all(np.abs(E - Eref) / np.diff(off) < 1e-6), (E, Eref)
    assert rel_rmse(F, Fref) < 1e-5
    m.close()


def test_batched_boxes_change_between_replays(P):
    """New boxes (and positions) every call: uploaded to device memory, the captured graph
    is replayed unchanged, and each call matches the oracle for its own boxes."""
    w = sy.model_weights(WATER, seed=1)
    pos, Z, off, boxes = _water_batch()
    m = P.NNPModel(WATER, weights=sy.flat_weights(w), precision="fp32")
    d = torch.from_numpy(pos).cuda()
    E = torch.empty(len(off) - 1, dtype=torch.float64, device="cuda")
    F = torch.empty((len(Z), 3), dtype=torch.float64, device="cuda")
    m.compute_batch(d, Z, off, boxes=boxes, out=(E, F))
    torch.cuda.synchronize()
    b0, u0, r0 = graph_counts(P, m)
    for k, s in enumerate((1.01, 1.025, 0.995)):
        scale = np.ones(len(Z), np.float32)
        bx = boxes.copy()
        for sys_i in range(3):   # the periodic systems grow or shrink with their boxes
            scale[off[sys_i]:off[sys_i + 1]] = s
            bx[sys_i] *= s
        p2 = (pos * scale[:, None]).astype(np.float32)
        d.copy_(torch.from_numpy(p2))
        m.compute_batch(d, None, off, boxes=bx, out=(E, F))
        torch.cuda.synchronize()
        junk = torch.randn(4096, device="cuda").sum().item()   # unrelated eager work between replays
        assert m.status() == 0
        Eref, Fref = orc.evaluate_batch(p2, Z, off, WATER, w, boxes=bx)
        assert np.all(np.abs(E.cpu().numpy() - Eref) / np.diff(off) < 1e-6), k
        assert rel_rmse(F.cpu().numpy(), Fref) < 1e-5, k
    b1, u1, r1 = graph_counts(P, m)
    assert b1 == b0 and r1 == r0 + 3, (b0, u0, r0, b1, u1, r1)
    m.close()


def test_batched_box_errors(P):
    w = sy.model_weights(WATER, seed=1)
    pos, Z, off, boxes = _water_batch()
    m = P.NNPModel(WATER, weights=sy.flat_weights(w), precision="fp32")
    d = torch.from_numpy(pos).cuda()
    for bad, status in (([10.0, 12.42, 12.42], P._lib.NNP_EBOX), ([12.42, 0.0, 12.42], P._lib.NNP_EBOX),
                        ([np.nan, 12.42, 12.42], P._lib.NNP_EBOX)):
        bx = boxes.copy()
        bx[0] = bad
        with pytest.raises(P.NNPError) as ex:
            m.compute_batch(d, Z, off, boxes=bx)
        assert ex.value.status == status
    m.close()


# ------------------------------------ link atoms across the periodic boundary
def _cut_bonds(pos, idx, n_all, cutoff=1.6):
    d = np.linalg.norm(pos[:, None].astype(np.float64) - pos[None], axis=-1)
    inside = set(int(a) for a in idx)
    ml, mm = [], []
    for a in idx:
        for b in range(n_all):
            if b not in inside and d[a, b] < cutoff:
                ml.append(int(a))
                mm.append(b)
    return np.array(ml, np.int32), np.array(mm, np.int32)


def _straddling_system():
    """A 30-atom H/C/N/O walk in a 44 A box; the first 18 atoms are the ML group.  The whole
    system is translated so that the first cut bond's midpoint lies on the x = 0 face, then
    every atom is wrapped into [0, L): the cut bond's two atoms sit at opposite faces."""
    rng = np.random.Generator(np.random.PCG64(21))
    pos, Z = sy.walk_molecule(30, rng)
    L = np.full(3, 44.0, np.float32)
    idx = np.arange(18, dtype=np.int32)
    ml, mm = _cut_bonds(pos, idx, 30)
    p = pos.astype(np.float64)
    mid = 0.5 * (p[ml[0]] + p[mm[0]])
    moved = p + np.array([-mid[0], 3.7 - mid[1], 5.1 - mid[2]])
    wrapped = (moved - 44.0 * np.floor(moved / 44.0)).astype(np.float32)
    assert abs(float(wrapped[ml[0], 0]) - float(wrapped[mm[0], 0])) > 22.0
    return wrapped, Z, L, idx, ml, mm


def test_link_atoms_across_periodic_boundary(P):
    w = sy.model_weights(HCNO, seed=1)
    pos, Z, L, idx, ml, mm = _straddling_system()
    ref = orc.evaluate(pos, Z, HCNO, w, box=L, nnp_idx=idx, links=(ml, mm, 1.0, 1))
    n_nnp = idx.size + ml.size
    d = torch.from_numpy(pos).cuda()
    # engine pair list over all atoms within the cutoff plus a buffer (half list, shuffled)
    I, J = orc.neighbour_pairs(pos, float(HCNO["rc_rad"]) + 0.5, L)
    keep = I < J
    pairs = np.stack([I[keep], J[keep]], axis=1).astype(np.int32)
    pairs = pairs[np.random.default_rng(4).permutation(len(pairs))]
    pairs_d = torch.from_numpy(np.ascontiguousarray(pairs)).cuda()
    for prec, tol_e, tol_f in (("fp32", 1e-6, 1e-5), ("bf16", 2e-3, 1e-2)):
        a = P.NNPModel(HCNO, weights=sy.flat_weights(w), precision=prec)
        b = P.NNPModel(HCNO, weights=sy.flat_weights(w), precision=prec)
        a.set_links(ml, mm, 1.0, 1)
        b.set_links(ml, mm, 1.0, 1)
        Ea, Fa, _ = a.compute(d, Z, L, nnp_idx=idx)
        Eb, Fb, _ = b.compute_pairs(d, pairs_d, Z, L, nnp_idx=idx)
        torch.cuda.synchronize()
        assert a.status() == 0 and b.status() == 0
        Fa_h = Fa.cpu().numpy()
        assert abs(Ea.item() - ref["E"]) / n_nnp < tol_e, (prec, Ea.item(), ref["E"])
        assert rel_rmse(Fa_h, ref["F"]) < tol_f, prec
        assert np.abs(Fa_h[mm]).max() > 0
        # the pair-list path builds the same lists (link atoms found by its direct scan)
        for buf in (P._lib.NNP_BUF_NBR_COUNT, P._lib.NNP_BUF_PERM):
            assert np.array_equal(a.read(buf), b.read(buf)), buf
        cnt = a.read(P._lib.NNP_BUF_NBR_COUNT)
        for buf, col in ((P._lib.NNP_BUF_NBR_RAD, 0), (P._lib.NNP_BUF_NBR_ANG, 1)):
            la, lb = a.read(buf), b.read(buf)
            mask = np.arange(la.shape[1])[None, :] < cnt[:, col][:, None]
            assert np.array_equal(np.where(mask, la, -1), np.where(mask, lb, -1)), buf
        assert Ea.item() == Eb.item()
        assert torch.equal(Fa, Fb)
        a.close()
        b.close()


# ---------------------------------------------------------- graph updates
def test_graph_update_on_box_change(P):
    """A box rescaled every call (as under a barostat): the captured graph is updated in
    place with the new box, never rebuilt, and each call equals direct launches."""
    w = sy.model_weights(WATER, seed=1)
    pos, Z, box = sy.water_box(64, 12.42, seed=0)
    m = P.NNPModel(WATER, weights=sy.flat_weights(w), precision="fp32")
    ref = P.NNPModel(WATER, weights=sy.flat_weights(w), precision="fp32")
    ref.set_graph(False)
    d = torch.from_numpy(pos).cuda()
    E = torch.empty(1, dtype=torch.float64, device="cuda")
    F = torch.empty((len(Z), 3), dtype=torch.float64, device="cuda")
    scales = (1.0, 1.004, 1.008, 1.012, 1.008, 1.008, 1.008)
    for k, s in enumerate(scales):
        d.copy_(torch.from_numpy((pos * np.float32(s)).astype(np.float32)))
        bk = (box * np.float32(s)).astype(np.float32)
        m.compute(d, Z if k == 0 else None, bk, out=(E, F, None))
        torch.cuda.synchronize()
        junk = torch.randn(2048, device="cuda").sum().item()   # unrelated eager work between calls
        Er, Fr, _ = ref.compute(d, Z if k == 0 else None, bk)
        torch.cuda.synchronize()
        assert E.item() == Er.item(), k
        assert torch.allclose(F, Fr, rtol=0, atol=1e-12), k
        if k in (0, len(scales) - 1):
            r = orc.evaluate((pos * np.float32(s)).astype(np.float32), Z, WATER, w, box=bk)
            assert rel_rmse(F.cpu().numpy(), r["F"]) < 1e-5
    builds, updates, replays = graph_counts(P, m)
    assert builds == 1 and updates == 4 and replays == 2, (builds, updates, replays)
    m.close()
    ref.close()


def test_autograd_path_replays(P):
    """Repeated NNPEnergy calls write into the model's persistent outputs and replay one
    graph; returned energies and gradients are independent copies."""
    w = sy.model_weights(WATER, seed=1)
    pos, Z, box = sy.water_box(64, 12.42, seed=0)
    m = P.NNPModel(WATER, weights=sy.flat_weights(w), precision="fp32")
    x = torch.from_numpy(pos).cuda()
    xk = torch.zeros_like(x).requires_grad_(True)   # an MD engine's position array, updated in place
    Es, Gs = [], []
    for k in range(4):
        with torch.no_grad():
            xk.copy_(x + 0.01 * k)
        xk.grad = None
        E = m.energy(xk, Z if k == 0 else None, box)
        E.backward()
        Es.append(E.detach().clone())
        Gs.append(xk.grad.clone())
    torch.cuda.synchronize()
    builds, updates, replays = graph_counts(P, m)
    assert builds == 1 and updates == 0 and replays == 3, (builds, updates, replays)
    for k in range(4):
        r = orc.evaluate((x + 0.01 * k).cpu().numpy(), Z, WATER, w, box=box)
        assert abs(Es[k].item() - r["E"]) / len(Z) < 1e-6, k
        assert rel_rmse(-Gs[k].double().cpu().numpy(), r["F"]) < 1e-5, k
    assert Es[0].item() != Es[1].item()
    m.close()
