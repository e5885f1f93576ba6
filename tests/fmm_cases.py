"""Shared helpers of the GPU parity tests: run the HIP FMM through the C ABI and the FP64 oracle."""
import numpy as np
import torch

from oracle import direct as od

G = 1.0
NU = 0.3
K = od.moduli(G, NU)


def to_dev(x):
    return None if x is None else torch.tensor(np.ascontiguousarray(x), dtype=torch.float64, device="cuda")


def run_fmm(src, nrm, w, a, b, kind, trg=None, precision=1, p=6, leaf_max=64, svd_eps=0.0, batch=None,
            batch_trg=None, return_plan=False, max_depth=0):
    from paper_1612_04082_amd import kfmm
    plan = kfmm.FmmPlan(to_dev(src), to_dev(nrm), to_dev(w), to_dev(trg), K=K, G=G, p=p, leaf_max=leaf_max,
                        precision=precision, svd_eps=svd_eps, batch_src=batch, batch_trg=batch_trg,
                        max_depth=max_depth)
    out = plan.eval(kind, to_dev(a), to_dev(b))
    torch.cuda.synchronize()
    res = out.cpu().numpy()
    if return_plan:
        return res, plan
    plan.close()
    return res


def run_oracle(src, nrm, w, a, b, kind, trg=None):
    t = src if trg is None else trg
    return od.direct(kind, t, src, w, a=a, b=b, nrm=nrm, K=K, G=G)


def rel_l2(x, ref):
    return float(np.linalg.norm(x - ref) / np.linalg.norm(ref))
