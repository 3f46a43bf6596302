"""Time-series analysis of FCIQMC output [Sec. 4].  TEST INFRASTRUCTURE.

* blocking analysis (Flyvbjerg-Petersen): the series is halved repeatedly by
  averaging neighbouring pairs (Eq. BlockingTransformation, Sec. 4.1); at
  every level the naive standard error sigma~(k)^2 = (mean(X'^2) - mean(X')^2)
  / Omega' is recorded, i.e. the biased variance over the block count, as the
  paper writes it.
* the plateau level is chosen by the M-test of Jonsson (2018), which tests
  whether the lag-1 autocovariances of all coarser levels vanish.  Reading:
  M_j = sum_{k >= j} n_k (gamma_k(1) / sigma_k^2)^2, compared with the
  chi-square quantile with (number of terms) degrees of freedom at the 99 %
  level; the smallest passing j is taken.
* shift estimator = blocked mean of the shift after `skip` steps (Sec. 4.2).
* ratio of means with linear error propagation using the blocked variances
  and covariance at the common blocking level (Sec. 4.2, reading).
* variational energy from replica shifts and overlaps (Sec. 4.3).  Reading:
  the shift and the overlap of the same step are paired.
"""
from dataclasses import dataclass

import numpy as np


@dataclass
class BlockingResult:
    mean: float
    err: float
    err_err: float
    k: int            # blocking level chosen (k - 1 transformations, as printed in the paper)
    blocks: int
    success: bool
    levels: list      # (blocks, sigma~(k)) per level


def _levels(x):
    x = np.asarray(x, dtype=np.float64)
    out = []
    while len(x) >= 2:
        n = len(x)
        mu = x.mean()
        var = np.mean(x * x) - mu * mu          # biased variance
        g1 = np.sum((x[:-1] - mu) * (x[1:] - mu)) / n
        out.append((n, var, g1))
        x = 0.5 * (x[0:n - n % 2:2] + x[1:n - n % 2:2])
    return out


def blocking_analysis(x, alpha=0.01):
    from scipy.stats import chi2
    x = np.asarray(x, dtype=np.float64)
    mean = float(x.mean())
    lv = _levels(x)
    d = len(lv)
    terms = np.array([n * (g / v) ** 2 if v > 0 else 0.0 for n, v, g in lv])
    chosen, ok = d - 1, False
    for j in range(d):
        Mj = terms[j:].sum()
        if Mj <= chi2.ppf(1 - alpha, d - j):
            chosen, ok = j, True
            break
    n, v, _ = lv[chosen]
    err = float(np.sqrt(v / n)) if v > 0 else 0.0
    err_err = err / np.sqrt(2.0 * max(n - 1, 1))
    ok = ok and n >= 16
    return BlockingResult(mean, err, err_err, chosen + 1, n, ok,
                          [(nn, float(np.sqrt(vv / nn)) if vv > 0 else 0.0) for nn, vv, _ in lv])


def shift_estimator(shift, skip=0):
    return blocking_analysis(np.asarray(shift)[skip:])


def _blocked(x, k):
    x = np.asarray(x, dtype=np.float64)
    for _ in range(k):
        n = len(x) - len(x) % 2
        x = 0.5 * (x[0:n:2] + x[1:n:2])
    return x


@dataclass
class RatioResult:
    ratio: float
    err: float
    k: int
    delta_y: float


def ratio_of_means(num, den, skip=0):
    """r = mean(num)/mean(den) with linear error propagation [Sec. 4.2]."""
    num = np.asarray(num, dtype=np.float64)[skip:]
    den = np.asarray(den, dtype=np.float64)[skip:]
    bx, by = blocking_analysis(num), blocking_analysis(den)
    k = max(bx.k, by.k) - 1
    X, Y = _blocked(num, k), _blocked(den, k)
    n = len(X)
    mx, my = X.mean(), Y.mean()
    vx = np.mean(X * X) - mx * mx
    vy = np.mean(Y * Y) - my * my
    cxy = np.mean(X * Y) - mx * my
    r = mx / my
    var_r = r * r * (vx / (n * mx * mx) + vy / (n * my * my) - 2.0 * cxy / (n * mx * my))
    return RatioResult(float(r), float(np.sqrt(max(var_r, 0.0))), k + 1,
                       float(np.sqrt(vy / n) / abs(my)))


def projected_energy(hproj, vproj, skip=0):
    return ratio_of_means(hproj, vproj, skip)


def variational_energy(shifts, overlaps, skip=0):
    """Variational energy from R replicas [Sec. 4.3, Eq.
    RayleighQuotientReplica with the Hamiltonian as the observable].

    shifts: (R, n) shift time series S_A^(n); overlaps: (P, n) time series
    c_A^(n) . c_B^(n) of the P = R(R-1)/2 pairs in the order A = 0.., then B.
    The numerator of pair (A, B) at step n is (S_A + S_B)/2 times its overlap
    at the same step; numerators and denominators are summed over pairs and
    the ratio of their means is taken with blocking.
    """
    S = np.asarray(shifts, dtype=np.float64)
    O = np.asarray(overlaps, dtype=np.float64)
    R = S.shape[0]
    pairs = [(a, b) for a in range(R) for b in range(a + 1, R)]
    if O.shape[0] != len(pairs):
        raise ValueError("variational_energy: need one overlap series per replica pair")
    num = np.zeros(S.shape[1])
    den = np.zeros(S.shape[1])
    for (a, b), o in zip(pairs, O):
        num += 0.5 * (S[a] + S[b]) * o
        den += o
    return ratio_of_means(num, den, skip)

