"""Learned sizing of threshold decompositions: pilot features -> MLP -> (k, p, q),
then the decomposition, an a-posteriori check and the adaptive fallback.

The paper fixes R_SVD and the oversampling by hand (section "Randomized
matrix decompositions"). For many independent channels with a threshold
rank, this module predicts per channel the rank k, the oversampling p and
the number of power steps q from the 16 pilot-sketch features, runs the
decomposition with l = k + p, and accepts it when

  * the rank rule did not hit the cap l - p (RANK_CAPPED clear), and
  * the computed spectrum says the kept values have converged for these
    (p, q): (s_l / s_k)^(4q + 2) <= 1e-8 (the subspace-iteration error
    factor of Halko et al. 2011 for the q-step scheme),

otherwise it runs the adaptive range finder (FP64) instead. All arithmetic on
matrices and on the network runs in the library's kernels; this module only
moves three numbers per channel between them.
"""

import math
from dataclasses import dataclass

P_GRID = (8, 16, 32, 64, 128, 192)
Q_MAX = 4
CONVERGED = 1e-8
# predicted ranks are inflated by 10 %: an under-predicted k fails the check
# (rank capped) and costs a fallback, an over-predicted one a few columns
K_MARGIN = 1.1


def standardize(T):
    """Column means and standard deviations of the raw targets (log10 k, p, q)."""
    import numpy as np
    T = np.asarray(T, dtype=np.float64)
    mu = T.mean(axis=0)
    sd = T.std(axis=0)
    sd[sd == 0] = 1.0
    return mu, sd


def targets_from_labels(labels):
    """(k, p, q) labels -> raw targets (log10 k, p, q)."""
    import numpy as np
    return np.array([[math.log10(k), p, q] for k, p, q in labels], dtype=np.float64)


def kpq_from_output(y, mu, sd, n):
    """Standardized network output -> (k, p, q): k with the K_MARGIN safety
    factor, rounded up and capped at n; p rounded up to the grid; q rounded
    up into 0..4."""
    raw = [float(y[i]) * sd[i] + mu[i] for i in range(3)]
    k = int(min(max(math.ceil(K_MARGIN * 10.0 ** raw[0]), 1), n))
    p = next((g for g in P_GRID if g >= raw[1]), P_GRID[-1])
    q = int(min(max(math.ceil(raw[2] - 1e-9), 0), Q_MAX))
    return k, p, q


@dataclass
class ChannelOutcome:
    rank: int
    S: object
    passes: int          # streams of A: pilot + main run (+ the fallback's)
    fell_back: bool
    predicted: tuple     # (k, p, q)
    reason: str = ""


def accept(S, rank, l, p, q, flags):
    """A-posteriori check of a threshold run sized by (k, p, q)."""
    from . import FLAG_JACOBI_MAXSWEEP, FLAG_RANK_CAPPED, FLAG_SYNC_TIMEOUT
    if flags & FLAG_SYNC_TIMEOUT:
        return False, "grid barrier timed out"
    if flags & FLAG_JACOBI_MAXSWEEP:
        return False, "small SVD not converged"
    if flags & FLAG_RANK_CAPPED:
        return False, "rank capped at l - p"
    if rank >= l:
        return True, "exact (l = min(m, n))"
    s_k, s_l = float(S[rank - 1]), float(S[l - 1])
    if s_k <= 0.0:
        return True, "zero spectrum"
    if (s_l / s_k) ** (4 * q + 2) > CONVERGED:
        return False, "kept values not converged"
    return True, "converged"


def decompose(A, net, mu, sd, tau, seed, channel, symmetric=False, block=64, q_fallback=1,
              precision="fp64", pilot_work=None):
    """One channel: pilot -> MLP -> threshold run -> check -> adaptive fallback.
    Returns (ChannelOutcome, pilot workspace for reuse)."""
    from . import run, pilot_features
    m, n = A.shape
    f, pilot_work = pilot_features(A, seed=seed, channel=channel, work=pilot_work)
    y = net.forward(f.view(1, -1)).cpu().numpy()[0]
    k, p, q = kpq_from_output(y, mu, sd, min(m, n))
    out = run(A, k, p, q, seed=seed, channel=channel, symmetric=symmetric, rank_mode="rel_threshold",
              rank_param=tau, want_u=False, want_v=False, want_residual=False, precision=precision,
              trailing_hp=1)
    ok, why = accept(out.S_all.cpu().numpy(), out.rank, out.l, p, q, out.flags)
    passes = 1 + (2 * q + 2)
    if ok:
        return ChannelOutcome(out.rank, out.S, passes, False, (k, p, q), why), pilot_work
    ad = run(A, 0, p, q_fallback, seed=seed, channel=channel, symmetric=symmetric,
             rank_mode="rel_threshold", rank_param=tau, adaptive=True, block=block,
             want_u=False, want_v=False, want_residual=False)
    passes += adaptive_passes(ad.blocks, q_fallback, ad.l, min(m, n))
    return ChannelOutcome(ad.rank, ad.S, passes, True, (k, p, q), why), pilot_work


def adaptive_passes(blocks, q, l, mn):
    """Streams of A used by the adaptive finder: per block 1 sketch + 2q power
    products + 1 projection, plus the stopping sketch unless the growth hit
    min(m, n)."""
    return blocks * (2 * q + 2) + (0 if l >= mn else 1)


def train_predictor(features, labels, epochs=300, batch=128, lr=3e-3, seed=0, device="cuda"):
    """Fit the MLP on (features N x 16, labels [(k, p, q)]) with Adam on the
    device. Labels should describe the spectrum alone (no cap at the channel
    size, which the features cannot see). Returns (net, mu, sd, final mean
    loss in standardized units)."""
    import numpy as np
    import torch
    from . import Mlp
    T = targets_from_labels(labels)
    mu, sd = standardize(T)
    Xd = torch.as_tensor(np.asarray(features, dtype=np.float32), device=device).contiguous()
    Td = torch.as_tensor(((T - mu) / sd).astype(np.float32), device=device).contiguous()
    net = Mlp(seed=seed, device=device)
    N = Xd.shape[0]
    last = []
    for ep in range(epochs):
        for b0 in range(0, N, batch):
            loss = net.train_step(Xd[b0:b0 + batch], Td[b0:b0 + batch], lr=lr)
            if ep == epochs - 1:
                last.append(loss)
    final = float(torch.cat(last).mean().item()) if last else float("nan")
    return net, mu, sd, final


def threshold_rank(n, d, tau):
    """Exact threshold rank of the constructed spectrum exp(-i/d) (capped at n)."""
    return min(n, 1 + int(math.floor(d * math.log(1.0 / tau))))
