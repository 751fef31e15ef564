"""Brute-force references used to pin the oracle on tiny inputs.

These enumerate every one of the N^T hidden state paths, so they share no
structure with the recursions they check: P(y) is the sum over paths of
pi_{q1} b_{q1}(y_1) prod_t a_{q_{t-1} q_t} b_{q_t}(y_t) (section 3.1 definitions).
"""
import itertools

import numpy as np
from scipy.special import logsumexp


def path_logps(log_pi, log_A, logB):
    T, n = logB.shape
    paths = np.array(list(itertools.product(range(n), repeat=T)), dtype=np.int64)
    lp = log_pi[paths[:, 0]] + logB[0, paths[:, 0]]
    for t in range(1, T):
        lp = lp + log_A[paths[:, t - 1], paths[:, t]] + logB[t, paths[:, t]]
    return paths, lp


def brute_posteriors(log_pi, log_A, logB):
    """Returns (logL, gamma [T,N], xi [T-1,N,N])."""
    T, n = logB.shape
    paths, lp = path_logps(log_pi, log_A, logB)
    logL = logsumexp(lp)
    w = np.exp(lp - logL)
    gamma = np.zeros((T, n))
    xi = np.zeros((max(T - 1, 0), n, n))
    for t in range(T):
        np.add.at(gamma[t], paths[:, t], w)
    for t in range(T - 1):
        np.add.at(xi[t], (paths[:, t], paths[:, t + 1]), w)
    return logL, gamma, xi


def brute_viterbi(log_pi, log_A, logB):
    paths, lp = path_logps(log_pi, log_A, logB)
    k = int(np.argmax(lp))
    return paths[k].astype(np.int32), float(lp[k]), np.sort(lp)[::-1]
