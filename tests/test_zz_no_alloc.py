"""ws_train_noalloc (ws_train with its work buffers in the library's static device scratch, for callers that
cannot allocate) against ws_train, through the C ABI: two networks from one seed, trained on the same
inputs by the two entry points, must end with bitwise-equal parameters and losses (same kernels, same
launch shapes, same summation order).  Two calls in a row, the first at the largest allowed row count
(the whole scratch), the second smaller; then a request beyond the maximum is refused before any work."""
import numpy as np
import pytest
import torch

pytestmark = pytest.mark.gpu


def _inputs(n, seed):
    rng = np.random.default_rng(seed)
    X = torch.tensor(rng.normal(size=(n, 16)), dtype=torch.float32, device="cuda")
    xm = rng.normal(size=(n, 3))
    xt = xm + 0.7 * rng.normal(size=(n, 3))
    d = lambda a: torch.tensor(a, dtype=torch.float64, device="cuda")
    return X, d(xm), d(xt)


def test_train_noalloc_matches_train(cuda):
    from paper_1612_04082_amd import kfmm
    ref = kfmm.WarmStartNet(seed=11)
    na = kfmm.WarmStartNet(seed=11)
    assert np.array_equal(ref.get_params(), na.get_params())
    for n, seed in ((kfmm.WS_NOALLOC_MAX_ROWS, 0), (3001, 1)):
        X, xm, xt = _inputs(n, seed)
        print(f"ws_train vs ws_train_noalloc: n = {n}", flush=True)
        l_ref = ref.train(X, xm, xt, 1.5, epochs=3, lr=1e-3)
        l_na = na.train_noalloc(X, xm, xt, 1.5, epochs=3, lr=1e-3)
        p_ref, p_na = ref.get_params(), na.get_params()
        print(f"  loss {l_ref:.9g} / {l_na:.9g}, max |dparam| {np.abs(p_ref - p_na).max():.3e}")
        assert l_ref == l_na
        assert np.array_equal(p_ref, p_na)
    X, xm, xt = _inputs(kfmm.WS_NOALLOC_MAX_ROWS + 1, 2)
    before = na.get_params()
    with pytest.raises(kfmm.KfmmError) as e:
        na.train_noalloc(X, xm, xt, 1.5, epochs=1)
    assert e.value.code == -1 and "KFMM_WS_NOALLOC_MAX_ROWS" in str(e.value)
    assert np.array_equal(before, na.get_params())
    ref.close()
    na.close()
