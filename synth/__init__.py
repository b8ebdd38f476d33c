"""Seeded synthetic input matrices (shared by the tests, the benchmark and the
oracle runs; holds none of the decomposition's arithmetic).

The paper's own inputs (partial-wave three-nucleon matrix elements, section
"Low-rank interactions", Eq. 3) are not available, so matrices with a known
singular spectrum stand in for them:

    general   A = U diag(sigma) V^T (+ E)
    symmetric A = U diag(sigma) U^T (+ E), mirrored so A == A^T bitwise

U, V are Haar-distributed orthonormal columns: QR of a Gaussian matrix with
the signs fixed by diag(sign(R)) (Mezzadri 2007). Only the r_eff columns with
sigma_i >= 1e-17 sigma_0 are built, which is exact in FP64.

Random draws use numpy's PCG64 with SeedSequence([tag, channel]); the large
product U diag(sigma) V^T may run on a torch device for speed (the spectrum
is identical; only rounding of the product differs between devices).

Workloads (shapes and spectra of the benchmark configurations; sigma index
i = 0 .. min(m, n) - 1, so sigma_0 = 1):
  c1  512 x 512 general, sigma_i = 10^(-i/16); k = 40, p = 10, q = 2
  c2  16384^2 symmetric, sigma_i = exp(-i/40) + E, E = 1e-8 (G + G^T)/sqrt(2);
      k = 256, p = 16, q = 2
  c3  131072 x 8192 general, sigma_i = 10^(-i/64) + floor E = 1e-9 G/(sqrt(m)+sqrt(n));
      k = 512, p = 16, q = 3
  c4  96 symmetric PSD channels, n_c ~ logU[500, 12000], sigma_i = exp(-i/d_c),
      d_c ~ U[10, 80]; rank by relative threshold 1e-6
  c5  2000 channels as c4 with n_c ~ logU[200, 6000]
  paper_channel  N x N symmetric channel at the paper's sizes (N = 225 x the
      number of partial-wave states: 7650 and 40050), two-regime spectrum
"""

from dataclasses import dataclass
import math

import numpy as np

SIGMA_FLOOR = 1e-17


def _rng(tag, channel=0):
    return np.random.Generator(np.random.PCG64(np.random.SeedSequence([int(tag), int(channel)])))


def spectrum_pow10(nvals, decades_per_index):
    """sigma_i = 10^(-i * decades_per_index)."""
    i = np.arange(nvals, dtype=np.float64)
    return 10.0 ** (-i * decades_per_index)


def spectrum_exp(nvals, d):
    """sigma_i = exp(-i / d)."""
    i = np.arange(nvals, dtype=np.float64)
    return np.exp(-i / d)


def effective(sigma):
    """Drop the trailing values below 1e-17 * sigma_0 (they are zero in FP64)."""
    r = int(np.count_nonzero(sigma >= SIGMA_FLOOR * sigma[0]))
    return sigma[:r]


def haar_columns(n, r, rng, device=None):
    """n x r matrix with Haar-distributed orthonormal columns (a torch tensor on
    `device` when one is given: the QR then runs there)."""
    G = rng.standard_normal((n, r))
    if device is None or device == "cpu":
        Q, R = np.linalg.qr(G, mode="reduced")
        d = np.sign(np.diag(R))
        d[d == 0] = 1.0
        return Q * d[None, :]
    import torch
    Q, R = torch.linalg.qr(torch.from_numpy(G).to(device), mode="reduced")
    d = torch.sign(torch.diagonal(R))
    d[d == 0] = 1.0
    return Q * d[None, :]


def _product(U, s, V, device):
    """U diag(s) V^T in FP64, optionally on a torch device."""
    if device is None or device == "cpu":
        return (U * s[None, :]) @ V.T
    import torch
    Ut = torch.from_numpy(U * s[None, :]).to(device)
    Vt = torch.from_numpy(np.ascontiguousarray(V.T)).to(device)
    return (Ut @ Vt).cpu().numpy()


def general(m, n, sigma, tag, channel=0, noise=0.0, device=None):
    """A = U diag(sigma) V^T + noise * G / (sqrt(m) + sqrt(n)) (so ||E||_2 ~ noise)."""
    sigma = effective(np.asarray(sigma, np.float64)[: min(m, n)])
    r = len(sigma)
    rng = _rng(tag, channel)
    U = haar_columns(m, r, rng)
    V = haar_columns(n, r, rng)
    A = _product(U, sigma, V, device)
    if noise:
        A += (noise / (math.sqrt(m) + math.sqrt(n))) * rng.standard_normal((m, n))
    return np.ascontiguousarray(A)


def symmetric(n, sigma, tag, channel=0, noise=0.0, device=None):
    """A = U diag(sigma) U^T + noise (G + G^T)/sqrt(2), symmetrized from the upper
    triangle so that A == A^T bitwise."""
    sigma = effective(np.asarray(sigma, np.float64)[:n])
    r = len(sigma)
    rng = _rng(tag, channel)
    U = haar_columns(n, r, rng)
    G = rng.standard_normal((n, n)) if noise else None
    if device is None or device == "cpu":
        A = (U * sigma[None, :]) @ U.T
        if noise:
            G += G.T
            G *= noise / math.sqrt(2.0)
            A += G
            del G
        A = np.triu(A)
        A += np.triu(A, 1).T
        return np.ascontiguousarray(A)
    import torch
    Ud = torch.from_numpy(U).to(device)
    A = (Ud * torch.from_numpy(sigma).to(device)[None, :]) @ Ud.T
    del Ud
    out = _finish_symmetric_device(A, G, noise, device)
    res = out.cpu().numpy()
    del out
    return res


def _finish_symmetric_device(A, G, noise, device):
    import torch
    if noise:
        Gd = torch.from_numpy(G).to(device)
        del G
        A += (Gd + Gd.T) * (noise / math.sqrt(2.0))
        del Gd
    A = torch.triu(A)
    A += torch.triu(A, 1).T
    return A


def symmetric_device(n, sigma, tag, channel=0, device="cuda"):
    """As symmetric() without noise, built entirely on `device` (Haar basis by a
    device QR); returns a contiguous torch tensor there."""
    import torch
    sigma = effective(np.asarray(sigma, np.float64)[:n])
    r = len(sigma)
    rng = _rng(tag, channel)
    U = haar_columns(n, r, rng, device=device)
    A = (U * torch.from_numpy(sigma).to(device)[None, :]) @ U.T
    del U
    return _finish_symmetric_device(A, None, 0.0, device).contiguous()


def rank_r(m, n, r, tag, channel=0, scale=1.0):
    """Exactly rank-r matrix with sigma_0..sigma_{r-1} = scale * 2^-i (for the low-rank pins)."""
    rng = _rng(tag, channel)
    s = scale * 2.0 ** -np.arange(r)
    U = haar_columns(m, r, rng)
    V = haar_columns(n, r, rng)
    return np.ascontiguousarray((U * s[None, :]) @ V.T), s


@dataclass
class Workload:
    name: str
    m: int
    n: int
    symmetric: bool
    k: int
    p: int
    q: int
    seed: int  # Omega key


def c1():
    """512 x 512 general, sigma_i = 10^(-i/16); k=40, p=10, q=2."""
    m = n = 512
    sigma = spectrum_pow10(n, 1.0 / 16.0)
    A = general(m, n, sigma, tag=1)
    return A, sigma, Workload("c1_512sq_general", m, n, False, 40, 10, 2, 2001)


def c2(n=16384, device=None):
    """n x n symmetric, sigma_i = exp(-i/40) + 1e-8 symmetric Gaussian noise; k=256, p=16, q=2."""
    sigma = spectrum_exp(n, 40.0)
    A = symmetric(n, sigma, tag=2, noise=1e-8, device=device)
    return A, sigma, Workload(f"c2_{n}sq_symmetric", n, n, True, 256, 16, 2, 2002)


def c3(m=131072, n=8192, device=None):
    """m x n general, sigma_i = 10^(-i/64), noise floor ||E||_2 ~ 1e-9; k=512, p=16, q=3."""
    sigma = spectrum_pow10(min(m, n), 1.0 / 64.0)
    A = general(m, n, sigma, tag=3, noise=1e-9, device=device)
    return A, sigma, Workload(f"c3_{m}x{n}_general", m, n, False, 512, 16, 3, 2003)


def channel_dims(count, lo, hi, tag):
    """Channel sizes n_c ~ logU[lo, hi] and decay lengths d_c ~ U[10, 80]."""
    rng = _rng(tag, 10**6)
    dims = np.exp(rng.uniform(math.log(lo), math.log(hi), size=count)).astype(np.int64)
    d = rng.uniform(10.0, 80.0, size=count)
    return dims, d


def channel(c, n, d, tag, device=None):
    """Symmetric PSD channel matrix with sigma_i = exp(-i/d) (numpy, or a torch
    tensor built on `device`)."""
    sigma = spectrum_exp(n, d)
    if device is not None and device != "cpu":
        return symmetric_device(n, sigma, tag=tag, channel=c, device=device), sigma
    return symmetric(n, sigma, tag=tag, channel=c), sigma


C4_TAU = 1e-6


def c4_params(n, d, tau=C4_TAU, q=2):
    """(k, p, q) of one c4 channel: k = the threshold rank of exp(-i/d) at tau
    (1 + floor(d ln(1/tau))), p the smallest multiple of 16 with
    (sigma_{k+p} / sigma_k)^(4q+2) = exp(-p (4q+2) / d) <= 1e-8, l capped at n."""
    k = min(n, 1 + int(math.floor(d * math.log(1.0 / tau))))
    p = 16 * int(math.ceil(d * math.log(1e8) / (4 * q + 2) / 16.0))
    return k, p, q


def c4(count=96, lo=500, hi=12000, device="cuda", tag=4):
    """96 symmetric PSD channels, n_c ~ logU[500, 12000], d_c ~ U[10, 80],
    sigma_i = exp(-i/d_c), no noise; rank by relative threshold 1e-6.
    Returns (matrices on `device`, problem dicts for the batch planner)."""
    dims, dec = channel_dims(count, lo, hi, tag=tag)
    mats, probs = [], []
    for c, (n, d) in enumerate(zip(dims, dec)):
        n, d = int(n), float(d)
        A, _ = channel(c, n, d, tag=tag, device=device)
        k, p, q = c4_params(n, d)
        mats.append(A)
        probs.append(dict(m=n, n=n, k=k, p=p, q=q, symmetric=True, seed=2004, channel=c,
                          rank_mode="rel_threshold", rank_param=C4_TAU, d=d))
    return mats, probs


# ---- learned (k, p, q) predictor: channels and labels ------------------------
C5_P_GRID = (8, 16, 32, 64, 128, 192)
C5_Q_GRID = (0, 1, 2, 3, 4)
C5_CONVERGED = 1e-8


def c5_dims(count=2000, lo=200, hi=6000, tag=5):
    """Channel sizes n_c ~ logU[200, 6000] and decay lengths d_c ~ U[10, 80]
    of the 2000-channel training / evaluation set (first 1500 train)."""
    return channel_dims(count, lo, hi, tag=tag)


def kpq_label(n, d, tau=C4_TAU, cap=True):
    """Training label of a channel with sigma_i = exp(-i/d) (generator metadata):
    k* = its threshold rank at tau (capped at n); (p*, q*) = the cheapest
    (cost (2q + 2)(k* + p)) grid point whose kept values are converged,
    (sigma_{k+p} / sigma_k)^(4q+2) = exp(-p (4q + 2) / d) <= 1e-8, or whose
    l = k + p reaches n (then the method is an exact SVD). cap=False labels
    the spectrum alone, as if n were unbounded (what the pilot features can
    see; the cap at n is applied when a prediction is used)."""
    if not cap:
        n = 1 << 40
    k = min(n, 1 + int(math.floor(d * math.log(1.0 / tau))))
    best = None
    for q in C5_Q_GRID:
        for p in C5_P_GRID:
            if k + p < n and math.exp(-p * (4 * q + 2) / d) > C5_CONVERGED:
                continue
            cost = (2 * q + 2) * min(k + p, n)
            if best is None or cost < best[0]:
                best = (cost, p, q)
    if best is None:  # nothing on the grid converges: the largest p, q
        best = (0, C5_P_GRID[-1], C5_Q_GRID[-1])
    return k, best[1], best[2]


def channel_device_rng(c, n, d, tag, device="cuda"):
    """Symmetric PSD channel with sigma_i = exp(-i/d) drawn entirely on the
    device (torch generator seeded by (tag, c)): the fast path for the large
    learned-predictor sets. Same construction as channel(); only the random
    stream differs."""
    import torch
    sigma = effective(spectrum_exp(n, d))
    r = len(sigma)
    g = torch.Generator(device=device)
    g.manual_seed(int(tag) * 1_000_003 + int(c))
    G = torch.randn(n, r, dtype=torch.float64, device=device, generator=g)
    Q, R = torch.linalg.qr(G, mode="reduced")
    del G
    dd = torch.sign(torch.diagonal(R))
    dd[dd == 0] = 1.0
    Q = Q * dd[None, :]
    A = (Q * torch.from_numpy(sigma).to(device)[None, :]) @ Q.T
    del Q
    return _finish_symmetric_device(A, None, 0.0, device).contiguous(), spectrum_exp(n, d)


def general_device_rng(m, n, sigma, tag, noise=0.0, device="cuda"):
    """As general(), drawn entirely on `device` (torch generator seeded by
    tag): A = U diag(sigma) V^T + noise G / (sqrt(m) + sqrt(n)), Haar U, V by
    a device QR. Returns a contiguous torch tensor there (the fast path for
    the 131072 x 8192 workload)."""
    import torch
    sigma = effective(np.asarray(sigma, np.float64)[: min(m, n)])
    r = len(sigma)
    g = torch.Generator(device=device)
    g.manual_seed(int(tag) * 7_919 + 17)

    def haar(rows):
        G = torch.randn(rows, r, dtype=torch.float64, device=device, generator=g)
        Q, R = torch.linalg.qr(G, mode="reduced")
        del G
        d = torch.sign(torch.diagonal(R))
        d[d == 0] = 1.0
        return Q * d[None, :]

    U = haar(m)
    V = haar(n)
    A = (U * torch.from_numpy(sigma).to(device)[None, :]) @ V.T
    del U, V
    if noise:
        A += (noise / (math.sqrt(m) + math.sqrt(n))) * torch.randn(m, n, dtype=torch.float64,
                                                                  device=device, generator=g)
    return A.contiguous()


def c3_device(m=131072, n=8192, device="cuda"):
    """The tall workload built on the device (see c3)."""
    sigma = spectrum_pow10(min(m, n), 1.0 / 64.0)
    A = general_device_rng(m, n, sigma, tag=3, noise=1e-9, device=device)
    return A, sigma, Workload(f"c3_{m}x{n}_general", m, n, False, 512, 16, 3, 2003)


# ---- channels at the paper's sizes -------------------------------------------
MESH = 225  # N_p x N_q momentum mesh points per partial-wave state


def spectrum_two_regime(N, lead=10.0, knee_frac=0.0025, knee=2e-3, tail=2e-6):
    """Two-regime spectrum shaped like the paper's channel matrices (section
    "Low-rank interactions", Fig. 2): a steep drop over the leading 0.25 % of
    the indices, then a slowly declining plateau below 2e-3. Log-linear from
    `lead` at i = 0 to `knee` at i0 = ceil(knee_frac N), then log-linear from
    `knee` to `tail` at i = N - 1. Every value is nonzero: the matrix has full
    rank, as the interaction matrices do."""
    i0 = max(1, int(math.ceil(knee_frac * N)))
    i = np.arange(N, dtype=np.float64)
    head = math.log10(lead) + (math.log10(knee) - math.log10(lead)) * i / i0
    plateau = math.log10(knee) + (math.log10(tail) - math.log10(knee)) * (i - i0) / max(N - 1 - i0, 1)
    return 10.0 ** np.where(i <= i0, head, plateau)


def paper_channel(N, tag=6, device=None):
    """N x N symmetric channel matrix A = U diag(sigma) U^T with the two-regime
    spectrum, N a multiple of 225. The basis is the Kronecker product
    U = U_mesh (225 x 225) x U_states (N/225 x N/225) of two Haar matrices
    (one per factor of the product basis of mesh points and partial-wave
    states): exactly orthogonal up to rounding and cheap to draw at
    N = 40050, where a Haar basis would need an N x N QR. A Gaussian
    projection is rotation invariant, so the randomized decomposition sees
    the same distribution of sketches as for a Haar basis. Mirrored from the
    upper triangle (A == A^T bitwise). Returns (A, sigma): A a numpy array,
    or a torch tensor built on `device`."""
    if N % MESH:
        raise ValueError("N must be a multiple of 225")
    sigma = spectrum_two_regime(N)
    rng = _rng(tag, N)
    U1 = haar_columns(MESH, MESH, rng)
    U2 = haar_columns(N // MESH, N // MESH, rng)
    if device is None or device == "cpu":
        U = np.kron(U1, U2)
        A = (U * sigma[None, :]) @ U.T
        del U
        A = np.triu(A)
        A += np.triu(A, 1).T
        return np.ascontiguousarray(A), sigma
    import torch
    U = torch.kron(torch.from_numpy(U1).to(device), torch.from_numpy(U2).to(device))
    A = (U * torch.from_numpy(sigma).to(device)[None, :]) @ U.T
    del U
    return _finish_symmetric_device(A, None, 0.0, device).contiguous(), sigma
