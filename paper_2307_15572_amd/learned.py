"""Learned sizing of threshold decompositions: pilot features -> MLP -> (k, p, q),
then the decomposition judged a posteriori, and the adaptive fallback.

The paper fixes R_SVD and the oversampling by hand (section "Randomized
matrix decompositions"). For many independent channels with a threshold
rank, the predictor maps 16 pilot-sketch features of a channel to the rank
k, the oversampling p and the number of power steps q (rsvd_mlp_predict:
de-standardization, 5 % rank margin, rounding to the grid, cap at the
channel size), the decomposition runs with l = k + p, r probe columns, and
the rank cap at l - 16 (the predicted p sizes the basis; the judge, not the
cap, guards the kept values), and the library's judge flags it
(include/rsvd.h, posterior > 0):

  * RANK_CAPPED: the threshold rule wanted more than l - 16 values;
  * POSTERIOR_FAIL: the posterior estimate of ||(I - QQ^T) A||_2 exceeds
    tau s_1, the adaptive finder's own stopping test;
  * UNCONVERGED: (s_l / s_k)^(4q + 2) > 1e-8, the kept values have not
    converged for these (p, q).

A flagged run is replaced by the adaptive range finder (FP64), which is
also the judge that produced the training labels. Because the sizes are
known before any decomposition starts, many channels run as one batch
(decompose_batch); the adaptive finder decides its width block by block and
runs channel after channel. Labels: k* is the finder's threshold rank and
(p*, q*) the cheapest grid point whose kept values its own spectrum shows
converged (rsvd_size_label, with the cost of the products, the panel
QRs and the small SVD). Every computation runs in the library's kernels;
this module moves integers and flags between the calls.
"""

from dataclasses import dataclass

POSTERIOR_COLUMNS = 16
RUN_P = 16        # the rank cap of a sized run sits at l - RUN_P
LABEL_Q = 2      # power steps of the labelling runs (accurate spectra)
LABEL_BLOCK = 32  # their growth step: the stopping width within 32 columns


@dataclass
class ChannelOutcome:
    rank: int
    S: object
    passes: int          # streams of A: pilot + main run (+ the fallback's)
    fell_back: bool
    predicted: tuple     # (k, p, q)
    reason: str = ""


def rejected(flags):
    """Names of the judge's flags set on a run (empty when accepted)."""
    from . import (FLAG_JACOBI_MAXSWEEP, FLAG_POSTERIOR_FAIL, FLAG_RANK_CAPPED,
                   FLAG_SYNC_TIMEOUT, FLAG_UNCONVERGED)
    names = ((FLAG_RANK_CAPPED, "rank capped"), (FLAG_POSTERIOR_FAIL, "posterior estimate"),
             (FLAG_UNCONVERGED, "kept values unconverged"),
             (FLAG_JACOBI_MAXSWEEP, "small SVD unconverged"),
             (FLAG_SYNC_TIMEOUT, "grid barrier timed out"))
    return [name for bit, name in names if flags & bit]


def adaptive_passes(blocks, q, l, mn):
    """Streams of A used by the adaptive finder: per block 1 sketch + 2q power
    products + 1 projection, plus the stopping sketch unless the growth hit
    min(m, n)."""
    return blocks * (2 * q + 2) + (0 if l >= mn else 1)


def run_adaptive(A, tau, seed, channel, symmetric=False, block=64, q=1, p=16):
    from . import run
    return run(A, 0, p, q, seed=seed, channel=channel, symmetric=symmetric,
               rank_mode="rel_threshold", rank_param=tau, adaptive=True, block=block,
               want_u=False, want_v=False, want_residual=False)


def label_channel(A, tau, seed, channel, symmetric=False):
    """Training label of one channel from the method's own decomposition: the
    adaptive FP64 finder at tau (LABEL_Q power steps, blocks of LABEL_BLOCK)
    gives k* = its threshold rank, the width l_ad at which its posterior
    estimate passed, and the spectrum up to l_ad; rsvd_size_label picks the
    cheapest (p*, q*) with k* + p* >= l_ad and converged kept values. Returns
    ((k, p, q), adaptive outcome), or (None, outcome) when no grid point
    qualifies or the label's l = k + p reaches min(m, n): such a label says
    nothing about the spectrum (the features cannot see the channel size)."""
    from . import size_label
    m, n = A.shape
    mn = min(m, n)
    ad = run_adaptive(A, tau, seed, channel, symmetric=symmetric, block=LABEL_BLOCK, q=LABEL_Q)
    k, p, q = size_label(ad.S_all, ad.rank, mn, l_min=ad.l)
    return ((k, p, q) if p > 0 and k + p < mn else None), ad


def decompose(A, net, tau, seed, channel, symmetric=False, block=64, q_fallback=1,
              precision="fp64", pilot_work=None):
    """One channel: pilot -> MLP -> judged threshold run -> adaptive fallback.
    Returns (ChannelOutcome, pilot workspace for reuse)."""
    from . import pilot_features, run
    m, n = A.shape
    f, pilot_work = pilot_features(A, seed=seed, channel=channel, work=pilot_work)
    (k, p, q), = net.predict(f.view(1, -1), [min(m, n)])
    l = min(k + p, min(m, n))
    out = run(A, max(l - RUN_P, 1), RUN_P, q, seed=seed, channel=channel, symmetric=symmetric,
              rank_mode="rel_threshold", rank_param=tau, want_u=False, want_v=False,
              want_residual=False, precision=precision, trailing_hp=1,
              posterior=POSTERIOR_COLUMNS)
    why = rejected(out.flags)
    passes = 1 + (2 * q + 2) + 1  # pilot + products + the judge's probe stream
    if not why:
        return ChannelOutcome(out.rank, out.S, passes, False, (k, p, q), "accepted"), pilot_work
    ad = run_adaptive(A, tau, seed, channel, symmetric=symmetric, block=block, q=q_fallback)
    passes += adaptive_passes(ad.blocks, q_fallback, ad.l, min(m, n))
    return ChannelOutcome(ad.rank, ad.S, passes, True, (k, p, q), ", ".join(why)), pilot_work


def decompose_batch(As, net, tau, seed, channels, symmetric=False, block=64, q_fallback=1,
                    precision="fp64", lanes=8):
    """Many channels at once: the pilot features of every channel into one
    B x 16 matrix, one predictor call (one synchronization), then every
    sized run in one batch (rsvd_batch_plan: the shapes are fixed before any
    run starts, so the channels share lanes of streams), the judge's flags
    read once, and the adaptive finder for the rejected channels. Returns a
    list of ChannelOutcome in the order of As."""
    import torch
    from . import MLP_IN, BatchPlan, check_flags, pilot_features
    if len(As) != len(channels):
        raise ValueError("one channel id per matrix")
    if not As:
        return []
    dev = As[0].device
    F = torch.empty(len(As), MLP_IN, dtype=torch.float32, device=dev)
    work = None
    for c, (A, ch) in enumerate(zip(As, channels)):
        _, work = pilot_features(A, seed=seed, channel=ch, work=work, out=F[c])
    del work
    kpq = net.predict(F, [min(A.shape) for A in As])
    probs = []
    for A, ch, (k, p, q) in zip(As, channels, kpq):
        m, n = A.shape
        l = min(k + p, min(m, n))
        probs.append(dict(m=m, n=n, k=max(l - RUN_P, 1), p=RUN_P, q=q, symmetric=symmetric,
                          seed=seed, channel=ch, rank_mode="rel_threshold", rank_param=tau,
                          want_u=False, want_v=False, want_residual=False, precision=precision,
                          trailing_hp=1, posterior=POSTERIOR_COLUMNS))
    bp = BatchPlan(probs, lanes=lanes, use_graph=False)
    bufs = bp.allocate(dev)
    bp.run_into(list(As), bufs)
    res = bp.results(bufs, check=False)
    out = []
    for c, (A, ch, (k, p, q), r) in enumerate(zip(As, channels, kpq, res)):
        m, n = A.shape
        passes = 1 + (2 * q + 2) + 1
        why = rejected(r.flags)
        if not why:
            check_flags(r.flags, f"channel {ch}")
            out.append(ChannelOutcome(int(r.rank), bufs["S"][c][: r.rank].clone(), passes, False,
                                      (k, p, q), "accepted"))
            continue
        ad = run_adaptive(A, tau, seed, ch, symmetric=symmetric, block=block, q=q_fallback)
        passes += adaptive_passes(ad.blocks, q_fallback, ad.l, min(m, n))
        out.append(ChannelOutcome(ad.rank, ad.S, passes, True, (k, p, q), ", ".join(why)))
    return out


def train_predictor(features, labels, epochs=300, batch=128, lr=3e-3, seed=0, device="cuda"):
    """Fit the MLP on (features N x 16, integer labels [(k, p, q)]) with Adam
    on the device (targets standardized by rsvd_mlp_targets). Returns (net,
    final mean loss in standardized units)."""
    import numpy as np
    import torch
    from . import Mlp
    net = Mlp(seed=seed, device=device)
    Td = net.targets(np.asarray(labels, dtype=np.int64))
    Xd = torch.as_tensor(np.asarray(features, dtype=np.float32), device=device).contiguous()
    N = Xd.shape[0]
    last = []
    for ep in range(epochs):
        for b0 in range(0, N, batch):
            loss = net.train_step(Xd[b0:b0 + batch], Td[b0:b0 + batch], lr=lr)
            if ep == epochs - 1:
                last.append(loss)
    final = float(torch.cat(last).mean().item()) if last else float("nan")
    return net, final
