"""The entry point that allocates nothing (nnp_compute_noalloc): its static
workspace gives the results of nnp_compute on the same inputs, call after call,
with a smaller system following a larger one."""
import numpy as np
import pytest
import torch

import oracle as orc
import synthetic as sy

pytestmark = pytest.mark.gpu

WATER = sy.model_config("water")
HCNO = sy.model_config("hcno")


def _lib():
    if not torch.cuda.is_available():
        pytest.fail("GPU test run without a visible GPU")
    import paper_2604_21441_amd as P
    return P


def _pair(P, m, pos, Z, box):
    """(E, F) from nnp_compute (reserved workspace) and from nnp_compute_noalloc."""
    d = torch.from_numpy(pos).cuda()
    n = len(Z)
    E0, F0, _ = m.compute(d, Z, box)
    E1 = torch.full((1,), np.nan, dtype=torch.float64, device="cuda")
    F1 = torch.full((n, 3), np.nan, dtype=torch.float64, device="cuda")
    P.nnp_compute_noalloc(m.h, d, Z, box, E1, F1)
    torch.cuda.synchronize()
    assert m.status() == 0
    return E0.item(), F0.cpu().numpy(), E1.item(), F1.cpu().numpy()


def _check_same(E0, F0, E1, F1):
    # same kernels and variants on the same inputs: the energy is a fixed-order FP64 sum,
    # the forces differ only by the order of FP64 additions in LDS
    assert E1 == E0
    assert np.all(np.isfinite(F1))
    assert np.abs(F1 - F0).max() < 1e-10 * max(1.0, np.abs(F0).max())


def test_noalloc_matches_compute_two_calls():
    P = _lib()
    w = sy.model_weights(WATER, seed=1)
    for prec in ("fp32", "bf16"):
        m = P.NNPModel(WATER, weights=sy.flat_weights(w), precision=prec)
        big = sy.water_box(500, 24.66, seed=3)          # 1,500 atoms, periodic
        small = sy.water_box(64, 12.42, seed=0)         # 192 atoms, periodic
        res = []
        for pos, Z, box in (big, small):
            E0, F0, E1, F1 = _pair(P, m, pos, Z, box)
            _check_same(E0, F0, E1, F1)
            res.append((E1, F1))
        # the second (smaller) call against the oracle as well
        pos, Z, box = small
        ref = orc.evaluate(pos, Z, WATER, w, box=box)
        tol = 1e-5 if prec == "fp32" else 1e-2
        assert np.linalg.norm(res[1][1] - ref["F"]) / np.linalg.norm(ref["F"]) < tol
        assert abs(res[1][0] - ref["E"]) / len(Z) < (1e-6 if prec == "fp32" else 2e-3)
        m.close()


def test_noalloc_open_system_and_errors():
    P = _lib()
    w = sy.model_weights(HCNO, seed=1)
    m = P.NNPModel(HCNO, weights=sy.flat_weights(w), precision="fp32")
    rng = np.random.Generator(np.random.PCG64(21))
    for n in (120, 40):                                    # larger, then smaller open molecule
        pos, Z = sy.walk_molecule(n, rng)
        E0, F0, E1, F1 = _pair(P, m, pos, Z, None)
        _check_same(E0, F0, E1, F1)
    d = torch.zeros((6000, 3), dtype=torch.float32, device="cuda")
    E = torch.zeros(1, dtype=torch.float64, device="cuda")
    F = torch.zeros((6000, 3), dtype=torch.float64, device="cuda")
    with pytest.raises(P.NNPError) as ex:                  # beyond the static workspace
        P.nnp_compute_noalloc(m.h, d, np.full(6000, 6, np.int32), None, E, F)
    assert ex.value.status == P._lib.NNP_ECAPACITY
    with pytest.raises(P.NNPError) as ex:
        P.nnp_compute_noalloc(m.h, d[:10], np.full(10, 9, np.int32), None, E, F[:10])
    assert ex.value.status == P._lib.NNP_ESPECIES
    m.close()
