"""Seeded parameter vectors for the learned displacement proposal's network
(He-normal weights, small biases) in the library's flat layout: W1[32][4][3][3]
b1[32] W2[32][32][3][3] b2 W3 b3 W4 b4 Wh[3][512] bh[3]. A generator only: it
holds none of the network's arithmetic."""
import numpy as np

N_PARAMS = 30467
_CIN = (4, 32, 32, 32)


def proposal_params(seed, scale=1.0, head_scale=1.0):
    rng = np.random.default_rng(seed)
    parts = []
    for cin in _CIN:
        parts.append(rng.normal(0.0, scale * np.sqrt(2.0 / (cin * 9)), 32 * cin * 9))
        parts.append(rng.normal(0.0, 0.01, 32))
    parts.append(rng.normal(0.0, head_scale * np.sqrt(1.0 / 512), 3 * 512))
    parts.append(np.zeros(3))
    p = np.concatenate(parts)
    assert p.size == N_PARAMS
    return p.astype(np.float32)
