"""Matrix-core gather/scatter GEMM (every KIFMM translation) vs a plain FP64 reference.

Checks the MFMA operand layouts of v_mfma_{f64,f32}_16x16x4 and v_mfma_f32_16x16x32_f16 (split FP16) as
used by the library, the column gather (in), scatter (out), per-column scale, and the store / add / atomic
modes, on several tiles with a ragged last tile.
"""
import numpy as np
import pytest
import torch

pytestmark = pytest.mark.gpu


def _case(precision, mode, seed=0, n_ops=3, kernel=0, NC=192):
    from paper_1612_04082_amd import kfmm
    rng = np.random.default_rng(seed)
    n_box, ncols = 90, 150
    A = rng.normal(size=(n_ops, NC, NC))
    X = rng.normal(size=(n_box, NC))
    op = np.sort(rng.integers(0, n_ops, size=ncols))
    cin = rng.integers(0, n_box, size=ncols)
    if mode == 2:
        cout = rng.integers(0, 40, size=ncols)  # repeated destinations
    else:
        cout = rng.permutation(n_box)[:ncols % n_box] if ncols <= n_box else None
        ncols2 = min(ncols, n_box)
        op, cin = op[:ncols2], cin[:ncols2]
        cout = rng.permutation(n_box)[:ncols2]
    scale = rng.uniform(0.5, 2.0, size=len(op))
    Y0 = rng.normal(size=(n_box, NC))
    tdt = {0: torch.float64, 1: torch.float32, 3: torch.float32}[precision]
    ydt = torch.float64 if precision == 0 else torch.float32
    At = torch.tensor(A).to(tdt).cuda()
    Xt = torch.tensor(X).to(tdt).cuda()
    Yt = torch.tensor(Y0).to(ydt).cuda()
    kfmm.selftest_gemm(precision, At, Xt, Yt, op, cin, cout, scale, mode, kernel)
    # reference from the rounded inputs
    Ar = At.double().cpu().numpy()
    Xr = Xt.double().cpu().numpy()
    ref = Yt.new_tensor(Y0).double().cpu().numpy().copy()
    if mode == 0:
        for j in range(len(op)):
            ref[cout[j]] = 0.0
    for j in range(len(op)):
        ref[cout[j]] += scale[j] * (Ar[op[j]] @ Xr[cin[j]])
    got = Yt.double().cpu().numpy()
    err = np.abs(got - ref).max() / np.abs(ref).max()
    return err


@pytest.mark.parametrize("precision,tol", [(0, 1e-13), (1, 2e-6), (3, 2e-6)])
@pytest.mark.parametrize("mode", [0, 1, 2])
def test_gemm_matches_reference(cuda, precision, tol, mode):
    err = _case(precision, mode)
    print(f"precision={precision} mode={mode} rel err {err:.3e}")
    assert err < tol


@pytest.mark.parametrize("precision,tol", [(0, 1e-13), (1, 2e-6)])
@pytest.mark.parametrize("mode", [0, 1, 2])
@pytest.mark.parametrize("kernel", [2, 3, 4])
def test_gemm_kernels(cuda, precision, tol, mode, kernel):
    """Every FP64/FP32 kernel (split-K, LDS-tiled with one or two buffers) forced on the same launches."""
    err = _case(precision, mode, seed=7, kernel=kernel)
    print(f"precision={precision} mode={mode} kernel={kernel} rel err {err:.3e}")
    assert err < tol


@pytest.mark.parametrize("mode", [0, 2])
@pytest.mark.parametrize("kernel", [2, 3, 4])
def test_gemm_single_operator_wide_tiles(cuda, mode, kernel):
    """One operator for every column: the FP64 launch then uses the 128-column tiles."""
    err = _case(0, mode, seed=3, n_ops=1, kernel=kernel)
    assert err < 1e-13


@pytest.mark.parametrize("precision,tol,kernel", [(p, t, k) for p, t in ((0, 1e-13), (1, 2e-6)) for k in (0, 2, 3, 4)]
                         + [(3, 2e-6, 0)])
def test_gemm_128_row_blocks(cuda, precision, tol, kernel):
    """NC a multiple of 128 but not of 96 (the padding of p = 8 vectors, 888 -> 896): 128-row blocks
    in the tiled kernels, 64-row blocks in the split-K and split-FP16 kernels (the split-FP16 kernel has
    no selectable variants)."""
    for mode in (0, 2):
        err = _case(precision, mode, seed=11, kernel=kernel, NC=256)
        assert err < tol, (mode, err)


@pytest.mark.parametrize("mode", [0, 1, 2])
def test_split16_wide_tiles(cuda, mode):
    """Split FP16 at NC = 480 (the compressed M2L width): 160-row x 128-column workgroup tiles."""
    err = _case(3, mode, seed=5, NC=480)
    print(f"mode={mode} rel err {err:.3e}")
    assert err < 2e-6


@pytest.mark.parametrize("NC", [96, 192, 256, 384, 480, 896])
def test_split16_wide_range(cuda, NC):
    """Split-FP16 products with operators and vectors spanning many decades: operators 27 decades apart,
    vectors 20 decades apart, and inside each operator and vector entries spread over 4 decades (rows
    and components graded by 10^(-4 i / NC), inside the 2^-17 range of full split precision).  Every
    output element must carry an FP32-level error relative to its own |A| |x|, not to the largest entry
    of its operator or vector."""
    from paper_1612_04082_amd import kfmm
    rng = np.random.default_rng(21)
    n_ops, n_box, ncols = 4, 70, 300
    grade = 10.0 ** (-4.0 * np.arange(NC) / NC)
    A = rng.normal(size=(n_ops, NC, NC)) * (10.0 ** np.array([-15, -3, 4, 12]))[:, None, None]
    A *= grade[None, :, None]
    X = rng.normal(size=(n_box, NC)) * (10.0 ** rng.uniform(-10, 10, size=n_box))[:, None] * grade[None, :]
    X[3] = 0.0  # an all-zero vector
    op = np.sort(rng.integers(0, n_ops, size=ncols))
    cin = rng.integers(0, n_box, size=ncols)
    cout = np.arange(ncols)
    At = torch.tensor(A, dtype=torch.float32).cuda()
    Xt = torch.tensor(X, dtype=torch.float32).cuda()
    Yt = torch.zeros(ncols, NC, dtype=torch.float32).cuda()
    kfmm.selftest_gemm(3, At, Xt, Yt, op, cin, cout, None, 0)
    Ar, Xr = At.double().cpu().numpy(), Xt.double().cpu().numpy()
    got = Yt.double().cpu().numpy()
    worst = 0.0
    for j in range(ncols):
        ref = Ar[op[j]] @ Xr[cin[j]]
        bound = np.abs(Ar[op[j]]) @ np.abs(Xr[cin[j]])  # error scale of any summation order, per element
        if not bound.max() > 0:
            assert not got[j].any()
            continue
        worst = max(worst, (np.abs(got[j] - ref) / bound).max())
    print(f"NC={NC} worst error / (|A||x|) per element {worst:.2e}")
    assert worst < 2e-6


@pytest.mark.parametrize("NC,ncols,n_ops", [(896, 2000, 1), (896, 300, 8), (480, 300, 1), (192, 16500, 1),
                                            (256, 9000, 1)])
@pytest.mark.parametrize("mode", [0, 1])
def test_split16_translation_tiles(cuda, NC, ncols, n_ops, mode):
    """Split FP16 in the 64-column tiles of the translation passes, at launch sizes that take each kernel:
    the k-group, two-stage-prefetch variant below 512 workgroups (NC = 896 with 2,000 columns: 448
    workgroups of 64 rows; NC = 896 with 8 operators; NC = 480: 96-row blocks) and the plain kernel above
    (NC = 192 with 16,500 columns: 516 workgroups of 96 rows; NC = 256 with 9,000 columns: 564 of 64 rows);
    ragged last tiles, store, and add with per-column factors.  Per element the error must stay at FP32
    level relative to |A| |x| (plus |Y0| when adding)."""
    from paper_1612_04082_amd import kfmm
    rng = np.random.default_rng(31 + NC + ncols)
    n_box = 200
    A = rng.normal(size=(n_ops, NC, NC)).astype(np.float32)
    X = rng.normal(size=(n_box, NC)).astype(np.float32)
    op = np.sort(rng.integers(0, n_ops, size=ncols))
    cin = np.sort(rng.integers(0, n_box, size=ncols))
    cout = rng.permutation(ncols)
    Y0 = rng.normal(size=(ncols, NC)).astype(np.float32)
    scale = rng.uniform(0.5, 2.0, size=ncols) if mode == 1 else None  # per-column factors with add
    Yt = torch.tensor(Y0).cuda()
    kfmm.selftest_gemm(3, torch.tensor(A).cuda(), torch.tensor(X).cuda(), Yt, op, cin, cout, scale, mode, kernel=1)
    got = Yt.double().cpu().numpy()
    A64, X64 = A.astype(np.float64), X.astype(np.float64)
    worst = 0.0
    for o in range(n_ops):
        j = np.nonzero(op == o)[0]
        if not len(j):
            continue
        sj = scale[j][:, None] if scale is not None else 1.0
        prod = sj * (X64[cin[j]] @ A64[o].T)
        bound = sj * (np.abs(X64[cin[j]]) @ np.abs(A64[o]).T)
        ref = prod + (Y0[cout[j]] if mode == 1 else 0.0)
        if mode == 1:
            bound = bound + np.abs(Y0[cout[j]])
        worst = max(worst, (np.abs(got[cout[j]] - ref) / bound).max())
    print(f"NC={NC} ncols={ncols} ops={n_ops} mode={mode} worst error / (|A||x|) {worst:.2e}")
    assert worst < 2e-6
