"""Cross-entropy benchmarking and sampling from a set of probabilities, in
plain FP64 numpy -- TEST INFRASTRUCTURE (see oracle/__init__.py).

Definitions followed:
  cross_entropy     Eq. (cee): -(1/m) sum_j log p_U(x_j) over a sample x_1..x_m
  fidelity          Eq. (ae): alpha = (H_0 - S) / (H_0 - H(p_U)); in the
                    Porter-Thomas regime H_0 = log 2^n + gamma and
                    H(p_U) = log 2^n - 1 + gamma (App. B)
  set_entropy       App. C: for a uniformly chosen set T of t bitstrings,
                    -(2^n / t) sum_{j in T} p_j log p_j estimates H(U)
  sample_from_set   App. C: draw j from T with probability p_j / sum_k p_k
"""
import numpy as np

EULER_GAMMA = 0.57721566490153286061


def probabilities(amps) -> np.ndarray:
    a = np.asarray(amps).astype(np.complex128)
    return a.real ** 2 + a.imag ** 2


def porter_thomas_h0(n: int) -> float:
    """Cross entropy of an uncorrelated (uniform) sample with a Porter-Thomas output (App. B)."""
    return n * np.log(2.0) + EULER_GAMMA


def porter_thomas_entropy(n: int) -> float:
    """Entropy of a Porter-Thomas output distribution over 2^n bitstrings (App. B)."""
    return n * np.log(2.0) - 1.0 + EULER_GAMMA


def cross_entropy(p) -> float:
    """Eq. (cee) over the nonzero probabilities of the sample."""
    p = np.asarray(p, dtype=np.float64)
    nz = p[p > 0]
    return float(-np.mean(np.log(nz))) if len(nz) else float("nan")


def fidelity(ce: float, n: int, h0: float = None, h: float = None) -> float:
    """Eq. (ae); Porter-Thomas H_0 and H(p_U) unless given."""
    h0 = porter_thomas_h0(n) if h0 is None else h0
    h = porter_thomas_entropy(n) if h is None else h
    return (h0 - ce) / (h0 - h)


def set_entropy(p, n: int) -> float:
    """App. C: -(2^n / t) sum p log p over a uniformly chosen set (zeros contribute 0)."""
    p = np.asarray(p, dtype=np.float64)
    nz = p[p > 0]
    return float(-(2.0 ** n) / len(p) * np.sum(nz * np.log(nz)))


def xeb_stats(amps, n: int) -> np.ndarray:
    """The eight numbers qgm_xeb reports, from their definitions."""
    p = probabilities(amps)
    nz = p[p > 0]
    ce = cross_entropy(p)
    return np.array([np.sum(np.log(nz)), np.sum(nz), np.sum(nz * np.log(nz)), float(len(p) - len(nz)), ce,
                     fidelity(ce, n), set_entropy(p, n), (2.0 ** n) / len(p) * np.sum(nz)])


def sample_from_set(p, u) -> np.ndarray:
    """App. C: index j for each uniform u in [0, 1), the first j whose inclusive
    cumulative sum exceeds u times the total (the last index if none)."""
    c = np.cumsum(np.asarray(p, dtype=np.float64))
    j = np.searchsorted(c, np.asarray(u, dtype=np.float64) * c[-1], side="right")
    return np.minimum(j, len(c) - 1).astype(np.int64)
