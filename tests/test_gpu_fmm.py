"""Parity of the HIP KIFMM (fmm_plan / fmm_eval through the C ABI) with the FP64 direct-sum oracle.

  * one-leaf trees: the method reduces to the direct sum (near field only) -> FP64 rounding level;
  * the unit-sphere cloud of 4096 points (plain KIFMM check): FP64 error small and falling with p;
  * FP32 and split-FP16-M2L precisions at their stated tolerances;
  * stress targets distinct from the sources;
  * the double-layer jump identity evaluated through the FMM (int P = -I at interior targets).
"""
import numpy as np
import pytest
import torch

from oracle import direct as od
from tests.fmm_cases import rel_l2, run_fmm, run_oracle
from tests.quadrature import sphere_rule
from workloads import geometry as geo

pytestmark = pytest.mark.gpu


def _small_cloud(n=700, seed=7):
    rng = np.random.default_rng(seed)
    x = rng.normal(size=(n, 3))
    nrm = rng.normal(size=(n, 3)); nrm /= np.linalg.norm(nrm, axis=1)[:, None]
    return x, nrm, rng.uniform(0.5, 1.5, n), rng.normal(size=(n, 3)), rng.normal(size=(n, 3))


@pytest.mark.parametrize("kind", [od.DISP, od.STRESS])
@pytest.mark.parametrize("precision,tol", [(0, 1e-13), (1, 2e-6)])
def test_single_leaf_equals_direct_sum(cuda, kind, precision, tol):
    x, n, w, a, b = _small_cloud()
    got = run_fmm(x, n, w, a, b, kind, precision=precision, leaf_max=100000)
    ref = run_oracle(x, n, w, a, b, kind)
    err = rel_l2(got, ref)
    print(f"kind={kind} prec={precision} single-leaf rel err {err:.3e}")
    assert err < tol


def test_sphere_fp64_p_sweep(cuda):
    c = geo.sphere_cloud(4096, seed=1)
    ref = run_oracle(c["src"], c["nrm"], c["w"], c["a"], None, od.DISP)
    errs = {}
    for p in (4, 5, 6):
        got = run_fmm(c["src"], c["nrm"], c["w"], c["a"], None, od.DISP, precision=0, p=p)
        errs[p] = rel_l2(got, ref)
    print("sphere FP64 errors by p:", errs)
    assert errs[5] < errs[4] and errs[6] < errs[5]
    assert errs[6] < 1e-5


@pytest.mark.parametrize("precision,tol", [(1, 1e-4)])
def test_sphere_low_precision(cuda, precision, tol):
    c = geo.sphere_cloud(4096, seed=1)
    ref = run_oracle(c["src"], c["nrm"], c["w"], c["a"], c["a"][::-1].copy(), od.DISP)
    got = run_fmm(c["src"], c["nrm"], c["w"], c["a"], c["a"][::-1].copy(), od.DISP, precision=precision)
    err = rel_l2(got, ref)
    print(f"sphere prec={precision} rel err {err:.3e}")
    assert err < tol


@pytest.mark.parametrize("p,precision,tol", [(6, 0, 5e-4), (8, 0, 2e-5), (8, 1, 2e-5)])
def test_stress_at_separate_targets(cuda, p, precision, tol):
    """Stress of the single+double layer at interior targets (eq. stress_1 kernels D, S); the derivative
    kernel D on the equivalent densities needs a higher order than displacement for the same error."""
    c = geo.sphere_cloud(4096, seed=1)
    rng = np.random.default_rng(3)
    trg = rng.uniform(-0.6, 0.6, size=(3000, 3))
    b = rng.normal(size=c["src"].shape)
    ref = run_oracle(c["src"], c["nrm"], c["w"], c["a"], b, od.STRESS, trg=trg)
    got = run_fmm(c["src"], c["nrm"], c["w"], c["a"], b, od.STRESS, trg=trg, precision=precision, p=p)
    err = rel_l2(got, ref)
    print(f"stress p={p} prec={precision} rel err {err:.3e}")
    assert err < tol


def test_double_layer_jump_through_fmm(cuda):
    pts, nrm, w = sphere_rule(R=1.0, n_theta=64, n_phi=128)
    rng = np.random.default_rng(2)
    trg = rng.uniform(-0.4, 0.4, size=(500, 3))
    for k in range(3):
        b = np.zeros_like(pts); b[:, k] = 1.0
        got = run_fmm(pts, nrm, w, None, b, od.DISP, trg=trg, precision=0, p=8)
        e = np.zeros(3); e[k] = 1.0
        err = np.abs(got + e[None]).max()
        print(f"jump identity component {k}: max err {err:.3e}")
        assert err < 1e-5


@pytest.mark.parametrize("tol,slack", [(1e-7, 1.05), (1e-6, 1.5)])
def test_compressed_m2l(cuda, tol, slack):
    """Shared-basis M2L compression (FP32): the rank is reported and the error stays at the dense level
    (the far-field truncation at p = 8, ~3e-5 here with a random double layer on the sphere)."""
    from tests.fmm_cases import to_dev, K, G
    from paper_1612_04082_amd import kfmm
    c = geo.sphere_cloud(4096, seed=1)
    rng = np.random.default_rng(8)
    b = rng.normal(size=c["src"].shape)
    ref = run_oracle(c["src"], c["nrm"], c["w"], c["a"], b, od.DISP)
    dense = run_fmm(c["src"], c["nrm"], c["w"], c["a"], b, od.DISP, precision=1, p=8)
    plan = kfmm.FmmPlan(to_dev(c["src"]), to_dev(c["nrm"]), to_dev(c["w"]), K=K, G=G, p=8, leaf_max=64,
                        precision=1, m2l_tol=tol)
    got = plan.eval(od.DISP, to_dev(c["a"]), to_dev(b)).cpu().numpy()
    rank = plan.info()["m2l_rank"]
    plan.close()
    e_c, e_d = rel_l2(got, ref), rel_l2(dense, ref)
    print(f"m2l_tol {tol:.0e}: rank {rank} of 888, compressed err {e_c:.2e}, dense err {e_d:.2e}")
    assert 0 < rank < 888
    assert e_c <= slack * e_d + 1e-7 and e_c < 5e-5



@pytest.mark.parametrize("m2l_tol,p", [(0.0, 8), (3e-7, 8), (3e-7, 9)])
def test_split16_m2l_matches_fp32(cuda, m2l_tol, p):
    """Split-FP16 products (M2L, translations, pseudo-inverse factors; dense and compressed operators, and
    p = 9 where the coefficient vectors exceed 1024 values and the scaled split falls back to FP32): the
    result agrees with the FP32 evaluation to well below the method's error, and the error against the
    oracle stays at the FP32 level."""
    from tests.fmm_cases import to_dev, K, G
    from paper_1612_04082_amd import kfmm
    c = geo.sphere_cloud(4096, seed=1)
    rng = np.random.default_rng(9)
    b = rng.normal(size=c["src"].shape)
    ref = run_oracle(c["src"], c["nrm"], c["w"], c["a"], b, od.DISP)
    out = {}
    for prec in (kfmm.FP32, kfmm.FP32_M2L_SPLIT16):
        plan = kfmm.FmmPlan(to_dev(c["src"]), to_dev(c["nrm"]), to_dev(c["w"]), K=K, G=G, p=p, leaf_max=64,
                            precision=prec, m2l_tol=m2l_tol)
        out[prec] = plan.eval(od.DISP, to_dev(c["a"]), to_dev(b)).cpu().numpy()
        assert plan.info()["n_v_pairs"] > 0
        plan.close()
    d = rel_l2(out[kfmm.FP32_M2L_SPLIT16], out[kfmm.FP32])
    e32, e16 = rel_l2(out[kfmm.FP32], ref), rel_l2(out[kfmm.FP32_M2L_SPLIT16], ref)
    print(f"p {p} m2l_tol {m2l_tol:.0e}: split16 vs fp32 {d:.2e}, errors {e16:.2e} / {e32:.2e}")
    assert d < 1e-6
    assert e16 <= 1.02 * e32 + 1e-7


@pytest.mark.parametrize("leaf", [64, 512])
def test_split16_folded_and_unfolded_downward_pass(cuda, leaf):
    """Split FP16 with the compressed M2L applies a leaf's fd1 (first DC2DE factor) inside the U and L2L
    products that form its check potential, unless a leaf has an X list (then the check potential gets the X
    sources as well and the separate fd1 product runs).  Leaves of at most 64 targets lose their X pairs to
    the near field, so every leaf folds; leaves of up to 512 targets keep some.  Both forms against the FP32
    evaluation of the same tree and against the oracle.  Adaptive input: half the points uniform in a cube,
    half on a small sphere near one corner."""
    from tests.fmm_cases import to_dev, K, G
    from paper_1612_04082_amd import kfmm
    rng = np.random.default_rng(leaf)
    n = 8000
    d = rng.normal(size=(n // 2, 3))
    d /= np.linalg.norm(d, axis=1)[:, None]
    src = np.vstack([rng.uniform(size=(n // 2, 3)), 0.25 + 0.2 * d])
    nrm = rng.normal(size=(n, 3))
    nrm /= np.linalg.norm(nrm, axis=1)[:, None]
    w, a, b = rng.uniform(0.5, 1.5, n), rng.normal(size=(n, 3)), rng.normal(size=(n, 3))
    ref = run_oracle(src, nrm, w, a, b, od.DISP)
    out = {}
    for prec in (kfmm.FP32, kfmm.FP32_M2L_SPLIT16):
        plan = kfmm.FmmPlan(to_dev(src), to_dev(nrm), to_dev(w), K=K, G=G, p=8, leaf_max=leaf, precision=prec,
                            m2l_tol=3e-7)
        out[prec] = plan.eval(od.DISP, to_dev(a), to_dev(b)).cpu().numpy()
        leaf_x = bool((plan.target_lists() & 2).any())
        plan.close()
    assert leaf_x == (leaf == 512)
    dd = rel_l2(out[kfmm.FP32_M2L_SPLIT16], out[kfmm.FP32])
    e32, e16 = rel_l2(out[kfmm.FP32], ref), rel_l2(out[kfmm.FP32_M2L_SPLIT16], ref)
    print(f"leaf {leaf} (leaf X lists: {leaf_x}): split16 vs fp32 {dd:.2e}, errors {e16:.2e} / {e32:.2e}")
    assert dd < 1e-6
    assert e16 <= 1.02 * e32 + 1e-7  # the fold adds no error (the method's own is 2.4e-5 on this cloud at p = 8)


def test_fp64_compressed_m2l_matches_dense(cuda):
    """KFMM_FP64 with m2l_tol 1e-8: FP64 contractions on the compressed basis (rank 716 of 888, padded to
    768) with per-offset ranks, against the dense FP64 M2L and the oracle on the sphere at p = 8, both
    layers, displacement and stress; the two forms differ by rounding through the pseudo-inverse (a few
    1e-7), far below the method's error, and repeated products are the same bits."""
    from tests.fmm_cases import to_dev, K, G
    from paper_1612_04082_amd import kfmm
    c = geo.sphere_cloud(4096, seed=1)
    rng = np.random.default_rng(9)
    b = rng.normal(size=c["src"].shape)
    for kind in (od.DISP, od.STRESS):
        ref = run_oracle(c["src"], c["nrm"], c["w"], c["a"], b, kind)
        out = {}
        for tol in (0.0, 1e-8):
            plan = kfmm.FmmPlan(to_dev(c["src"]), to_dev(c["nrm"]), to_dev(c["w"]), K=K, G=G, p=8, leaf_max=64,
                                precision=kfmm.FP64, m2l_tol=tol)
            out[tol] = plan.eval(kind, to_dev(c["a"]), to_dev(b)).cpu().numpy()
            again = plan.eval(kind, to_dev(c["a"]), to_dev(b)).cpu().numpy()
            assert np.array_equal(out[tol], again)
            if tol > 0:
                assert plan.info()["m2l_rank"] == 768
            plan.close()
        d = rel_l2(out[1e-8], out[0.0])
        e0, e1 = rel_l2(out[0.0], ref), rel_l2(out[1e-8], ref)
        print(f"kind {kind}: compressed vs dense {d:.2e}, errors {e1:.2e} / {e0:.2e}")
        assert d < 2e-6 and e1 <= 1.05 * e0 + 1e-7


def test_profile_modes(cuda):
    """Phase timing (every phase in turn) and M2L-only timing leave the results bitwise unchanged."""
    from tests.fmm_cases import to_dev, K, G
    from paper_1612_04082_amd import kfmm
    c = geo.sphere_cloud(6000, seed=4)
    plan = kfmm.FmmPlan(to_dev(c["src"]), to_dev(c["nrm"]), to_dev(c["w"]), K=K, G=G, p=6, leaf_max=64,
                        precision=kfmm.FP32, m2l_tol=1e-6)
    a, b = to_dev(c["a"]), to_dev(c["a"][::-1].copy())
    ref = plan.eval(kfmm.DISP, a, b)
    plan.profile(True)
    got1 = plan.eval(kfmm.DISP, a, b)
    ph, n1 = plan.phase_times()
    plan.profile("m2l")
    for _ in range(3):
        got2 = plan.eval(kfmm.DISP, a, b)
    m2l, n2 = plan.phase_times()
    plan.profile(False)
    plan.close()
    assert torch.equal(ref, got1) and torch.equal(ref, got2)
    assert n1 == 1 and all(v >= 0 for v in ph.values()) and ph["m2l"] > 0
    assert n2 == 3 and m2l["m2l"] > 0 and all(v == 0 for k, v in m2l.items() if k != "m2l")


def test_fp32_trans64_matches_fp32(cuda):
    """FP32 M2L with FP64 pseudo-inverses and translations (KFMM_FP32_TRANS64, compressed M2L) against the
    FP32 translations on check potentials: both at the method's error, close to each other."""
    from tests.fmm_cases import to_dev, K, G
    from paper_1612_04082_amd import kfmm
    c = geo.sphere_cloud(4096, seed=1)
    rng = np.random.default_rng(10)
    b = rng.normal(size=c["src"].shape)
    ref = run_oracle(c["src"], c["nrm"], c["w"], c["a"], b, od.DISP)
    out = {}
    for prec in (kfmm.FP32, kfmm.FP32_TRANS64):
        plan = kfmm.FmmPlan(to_dev(c["src"]), to_dev(c["nrm"]), to_dev(c["w"]), K=K, G=G, p=8, leaf_max=64,
                            precision=prec, m2l_tol=3e-7)
        out[prec] = plan.eval(od.DISP, to_dev(c["a"]), to_dev(b)).cpu().numpy()
        plan.close()
    d = rel_l2(out[kfmm.FP32_TRANS64], out[kfmm.FP32])
    e32, e64 = rel_l2(out[kfmm.FP32], ref), rel_l2(out[kfmm.FP32_TRANS64], ref)
    print(f"trans64 vs fp32 translations {d:.2e}, errors {e64:.2e} / {e32:.2e}")
    assert d < 1e-6 and e64 < 5e-5 and e32 < 5e-5
