"""Product-basis sampling of an MPS, the collapse step of a METTS chain.

TEST INFRASTRUCTURE ONLY (see ``oracle/__init__``).

The paper's METTS chains start from product states sampled from the ground
state and alternate evolution with such collapses (Appendix D).  For a state
that is right-orthonormal with the centre on site 1, the probability of s_1
is ||A_1[:, s_1, :]||^2 / ||psi||^2 and, given s_1 .. s_(i-1) with left
vector v (normalised), the conditional probability of s_i is proportional to
||v A_i[:, s_i, :]||^2: the sites to the right are isometries.  A sample
draws s_i as the first s with P(s' <= s) > u and P(s) > 0 (u uniform in
[0, 1), supplied by the caller), then continues with v A_i[:, s_i, :]
normalised.

Pins (``tests/test_oracle_sampling.py``): the product of the conditional
probabilities of any configuration equals |psi(s)|^2 / ||psi||^2 from the
dense vector; basis product states are returned unchanged; the frequencies
of many samples follow |psi(s)|^2 within their statistical error.
"""
from __future__ import annotations

import numpy as np


def sample(psi, uniforms):
    """uniforms [L][S]; returns (configs [S][L], probabilities [S])."""
    L = len(psi)
    S = uniforms.shape[1]
    configs = np.zeros((S, L), dtype=np.int64)
    probs = np.ones(S)
    for k in range(S):
        v = np.ones(1)
        for i, A in enumerate(psi):
            t = np.einsum("a,asb->sb", v, A)
            p = np.sum(t * t, axis=1)
            tot = float(p.sum())
            thr = uniforms[i, k] * tot
            pick, cum = -1, 0.0
            for s in range(len(p)):
                cum += p[s]
                if pick < 0 and cum > thr and p[s] > 0.0:
                    pick = s
            if pick < 0:
                nz = np.nonzero(p > 0.0)[0]
                pick = int(nz[-1]) if len(nz) else 0
            configs[k, i] = pick
            probs[k] *= p[pick] / tot if tot > 0.0 else 0.0
            v = t[pick] / np.sqrt(p[pick]) if p[pick] > 0.0 else 0.0 * t[pick]
    return configs, probs
