"""Helpers for the GPU parity tests: move seeded inputs to the device and
results back.  Inputs come from paper_2311_06952_amd.synth (or numpy in the
test); expected values come only from the oracle."""
import numpy as np


def u32(t):
    """Device int32 tensor holding uint32 bits -> numpy uint32."""
    return t.cpu().numpy().view(np.uint32)


def np_(t):
    return t.cpu().numpy()


def dev(a, dtype=None):
    import torch
    a = np.ascontiguousarray(a)
    if a.dtype == np.uint32:
        a = a.view(np.int32)
    t = torch.as_tensor(a).cuda()
    return t if dtype is None else t.to(dtype)


def random_trees(rng, P, D, F, n_unique, p_nosplit=0.15, top=True):
    """Random (feat, tau) trees as inputs: feat in 0..F (0 with prob
    p_nosplit), tau in [0, n_f] for feat != 0 (the top value sends all left)."""
    SB = (1 << D) - 1
    feat = rng.integers(1, F + 1, size=(P, SB))
    feat[rng.random((P, SB)) < p_nosplit] = 0
    tau = np.zeros((P, SB), dtype=np.uint32)
    for r in range(P):
        for t in range(SB):
            f = feat[r, t]
            if f:
                hi = int(n_unique[f - 1]) + (1 if top else 0)
                tau[r, t] = rng.integers(0, hi)
    return feat.astype(np.uint8), tau
