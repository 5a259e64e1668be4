"""Comparison helpers for the parity tests (no arithmetic of the method)."""
import numpy as np


def gauge_fix(phi, mu):
    """Scaling vectors are unique only up to phi^k -> c_k phi^k with prod c_k = 1.
    Canonical representative: psi^k = phi^k exp(-mu^k . log phi^k) for k >= 1, and
    psi^0 = phi^0 prod_{k >= 1} exp(mu^k . log phi^k) (the plan K (.) Phi is unchanged)."""
    out = [np.array(p, dtype=np.float64) for p in phi]
    total = 0.0
    for k in range(1, len(out)):
        pos = mu[k] > 0
        g = float(np.sum(mu[k][pos] * np.log(out[k][pos])))
        out[k] = out[k] * np.exp(-g)
        total += g
    out[0] = out[0] * np.exp(total)
    return out


def max_rel(a_list, b_list):
    return max(float(np.max(np.abs(a - b) / np.abs(b))) for a, b in zip(a_list, b_list))


def rel_to_max(a, b):
    return float(np.max(np.abs(a - b)) / np.max(np.abs(b)))
