"""Batched plans (several independent geometries in one fmm_plan / fmm_eval): geometries never interact,
each has its own root, so a batched evaluation equals the per-geometry evaluations up to rounding, and
each matches the FP64 oracle on sampled targets.  Cells are periodic-cell bodies (unit cube minus
ellipsoids) that all occupy the same unit cube, so any interaction between them would be an O(1) change."""
import numpy as np
import pytest

from oracle import direct as od
from tests.fmm_cases import K, G, rel_l2, run_fmm
from workloads import geometry as geo

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def cells():
    return geo.cell_batch(6)


@pytest.mark.parametrize("precision", [1, 3])
def test_batched_equals_separate(cuda, cells, precision):
    """Launches of the batched plan are larger, so some translation products run on another kernel (tiled
    instead of split-K, or the k-split split-FP16 variant): the same sums grouped differently.  Two such
    evaluations differ by at most the sum of their rounding errors, each about the distance of the separate
    evaluation from the same plan in FP64, so the bound is 3x that distance (measured per geometry)."""
    src = np.concatenate([c["src"] for c in cells])
    nrm = np.concatenate([c["nrm"] for c in cells])
    w = np.concatenate([c["w"] for c in cells])
    a = np.concatenate([c["a"] for c in cells])
    b = np.concatenate([c["b"] for c in cells])
    off = np.concatenate([[0], np.cumsum([c["src"].shape[0] for c in cells])])
    got = run_fmm(src, nrm, w, a, b, od.DISP, precision=precision, p=6, leaf_max=128, batch=list(off))
    for g, c in enumerate(cells):
        one = run_fmm(c["src"], c["nrm"], c["w"], c["a"], c["b"], od.DISP, precision=precision, p=6, leaf_max=128)
        one64 = run_fmm(c["src"], c["nrm"], c["w"], c["a"], c["b"], od.DISP, precision=0, p=6, leaf_max=128)
        d = rel_l2(got[off[g]:off[g + 1]], one)
        e = rel_l2(one, one64)
        print(f"geometry {g}: batched vs separate {d:.2e}; separate vs FP64 {e:.2e}")
        assert d <= 3 * e, (g, d, e)


def test_batched_matches_oracle(cuda, cells):
    src = np.concatenate([c["src"] for c in cells])
    nrm = np.concatenate([c["nrm"] for c in cells])
    w = np.concatenate([c["w"] for c in cells])
    a = np.concatenate([c["a"] for c in cells])
    b = np.concatenate([c["b"] for c in cells])
    off = np.concatenate([[0], np.cumsum([c["src"].shape[0] for c in cells])])
    got = run_fmm(src, nrm, w, a, b, od.DISP, precision=1, p=8, leaf_max=128, batch=list(off))
    rng = np.random.default_rng(4)
    for g, c in enumerate(cells):
        idx = rng.choice(c["src"].shape[0], size=300, replace=False)
        ref = od.direct(od.DISP, c["src"][idx], c["src"], c["w"], a=c["a"], b=c["b"], nrm=c["nrm"], K=K, G=G)
        err = rel_l2(got[off[g]:off[g + 1]][idx], ref)
        print(f"cell {g}: {c['src'].shape[0]} points, rel err {err:.2e}")
        assert err < 2e-5


def test_batched_separate_targets(cuda, cells):
    """Batched plan with targets distinct from the sources (offsets for both)."""
    rng = np.random.default_rng(5)
    cs = cells[:3]
    src = np.concatenate([c["src"] for c in cs])
    nrm = np.concatenate([c["nrm"] for c in cs])
    w = np.concatenate([c["w"] for c in cs])
    a = np.concatenate([c["a"] for c in cs])
    trg = [rng.uniform(0.1, 0.9, size=(500 + 100 * g, 3)) for g in range(3)]
    off = list(np.concatenate([[0], np.cumsum([c["src"].shape[0] for c in cs])]))
    offt = list(np.concatenate([[0], np.cumsum([t.shape[0] for t in trg])]))
    got = run_fmm(src, nrm, w, a, None, od.STRESS, trg=np.concatenate(trg), precision=0, p=8, leaf_max=128,
                  batch=off, batch_trg=offt)
    for g, c in enumerate(cs):
        ref = od.direct(od.STRESS, trg[g], c["src"], c["w"], a=c["a"], nrm=c["nrm"], K=K, G=G)
        err = rel_l2(got[offt[g]:offt[g + 1]], ref)
        print(f"cell {g}: stress at {trg[g].shape[0]} targets, rel err {err:.2e}")
        assert err < 1e-4
