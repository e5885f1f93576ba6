"""Host-side logic of the Algorithm 1 harness (no GPU): post-processing keeps the material connected to
both end layers."""
import numpy as np

from paper_1612_04082_amd.alg1 import postprocess


def test_postprocess_keeps_connected_to_both_ends():
    M = np.zeros((6, 3, 3), bool)
    M[:, 1, 1] = True          # a bar from end to end
    M[2, 0, 0] = True          # floating voxel
    M[0:2, 2, 2] = True        # stub attached to one end only (not face-connected to the bar)
    out = postprocess(M)
    assert out[:, 1, 1].all()
    assert not out[2, 0, 0]
    assert not out[0:2, 2, 2].any()
    # cut bar: nothing connects both ends -> empty
    M2 = M.copy()
    M2[3, 1, 1] = False
    assert not postprocess(M2).any()
