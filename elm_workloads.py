"""Seeded synthetic ELM workloads.

This module only draws inputs: samples X (N x d), random hidden-node weights
W (d x L) and biases b (L), and targets T (N x m).  It computes nothing of the
method itself (no hidden layer, no Gram, no factorisation), so both the FP64
CPU oracle and the GPU path may use it without sharing any of the method's
arithmetic.

Random input weights and biases follow the ELM recipe of Section 2 (step 1 of
the three-step ELM, and step 1 of the RBP-ELM algorithm): w_j ~ U[-1, 1],
b_j ~ U[0, 1].  Rank deficiency is planted by duplicating hidden nodes: a
duplicated (w_j, b_j) pair gives a bitwise-identical column of H, so the rank
of H equals the number of distinct nodes whenever N is at least that number.

The paper's own datasets (OCRHD, GINA) are not available; the shapes below are
synthetic stand-ins with the structure of the workloads each one names.
"""
from __future__ import annotations

import dataclasses
import math
from typing import List, Optional

import numpy as np


@dataclasses.dataclass
class Problem:
    """One ELM training problem.

    X: (N, d) float64 samples, one per row.
    W: (d, L) float64 input-to-hidden weights, one hidden node per column.
    b: (L,)   float64 hidden biases.
    T: (N, m) float64 targets (one-hot rows for classification).
    labels: (N,) int class index for classification problems, else None.
    groups: (L,) int, for each hidden node the index of its distinct node
            (duplicated nodes share a group); n_distinct = groups.max() + 1.
    """
    name: str
    X: np.ndarray
    W: np.ndarray
    b: np.ndarray
    T: np.ndarray
    labels: Optional[np.ndarray]
    groups: np.ndarray

    @property
    def N(self) -> int:
        return self.X.shape[0]

    @property
    def d(self) -> int:
        return self.X.shape[1]

    @property
    def L(self) -> int:
        return self.W.shape[1]

    @property
    def m(self) -> int:
        return self.T.shape[1]

    @property
    def n_distinct(self) -> int:
        return int(self.groups.max()) + 1 if self.groups.size else 0

    @property
    def structural_rank(self) -> int:
        """Rank of H implied by the planted node duplication (generic X)."""
        return min(self.N, self.n_distinct)


def make_nodes(rng: np.random.Generator, d: int, L: int, n_dup: int):
    """L hidden nodes of which n_dup copy one of the L - n_dup distinct ones.

    Distinct nodes: w ~ U[-1,1]^d, b ~ U[0,1].  Each duplicate copies a
    distinct node chosen uniformly with replacement; the L columns are then
    shuffled so duplicates are scattered.
    """
    n_unique = L - n_dup
    if n_unique < 1:
        raise ValueError("need at least one distinct node")
    Wu = rng.uniform(-1.0, 1.0, size=(d, n_unique))
    bu = rng.uniform(0.0, 1.0, size=n_unique)
    src = np.concatenate([np.arange(n_unique), rng.integers(0, n_unique, size=n_dup)])
    perm = rng.permutation(L)
    groups = src[perm]
    W = np.ascontiguousarray(Wu[:, groups])
    b = np.ascontiguousarray(bu[groups])
    return W, b, groups.astype(np.int64)


def one_hot(labels: np.ndarray, m: int) -> np.ndarray:
    T = np.zeros((labels.shape[0], m), dtype=np.float64)
    T[np.arange(labels.shape[0]), labels] = 1.0
    return T


def tiny_fp64(seed: int = 1) -> Problem:
    """Plain FP64 ELM, tiny: N=2000, d=20, L=200 (40 duplicated nodes, rank 160),
    two one-hot classes from a random linear rule."""
    rng = np.random.default_rng(seed)
    N, d, L, n_dup = 2000, 20, 200, 40
    X = rng.uniform(-1.0, 1.0, size=(N, d))
    W, b, groups = make_nodes(rng, d, L, n_dup)
    v = rng.standard_normal(d)
    labels = (X @ v > 0).astype(np.int64)
    return Problem("tiny_fp64", X, W, b, one_hot(labels, 2), labels, groups)


def digits_like(seed: int = 2, N: int = 60000, L: int = 2000) -> Problem:
    """MNIST-like shape: N=60000, d=784 features in [0,1] with ~80% exact zeros,
    L=2000 distinct nodes (full rank), 10 classes by nearest of 10 centroids
    (centroids are 10 distinct rows of X)."""
    rng = np.random.default_rng(seed)
    d, m = 784, 10
    X = rng.uniform(0.0, 1.0, size=(N, d)) * (rng.uniform(0.0, 1.0, size=(N, d)) < 0.2)
    W, b, groups = make_nodes(rng, d, L, 0)
    cidx = rng.choice(N, size=m, replace=False)
    C = X[cidx]
    # nearest centroid by squared Euclidean distance, chunked to bound memory
    labels = np.empty(N, dtype=np.int64)
    cn = (C * C).sum(1)
    for s in range(0, N, 8192):
        xs = X[s:s + 8192]
        dist = cn[None, :] - 2.0 * xs @ C.T
        labels[s:s + 8192] = np.argmin(dist, axis=1)
    return Problem("digits_like", X, W, b, one_hot(labels, m), labels, groups)


def mixture_rankdef(seed: int = 3, N: int = 100000, L: int = 5000, dup_frac: float = 0.1) -> Problem:
    """Forest-cover-like shape: N=100000, d=54 from a 7-component Gaussian
    mixture (means N(0, 4I), unit variance), L=5000 nodes with 10% duplicated
    (rank 4500), 7 one-hot classes (the component)."""
    rng = np.random.default_rng(seed)
    d, m = 54, 7
    mu = 2.0 * rng.standard_normal((m, d))
    comp = rng.integers(0, m, size=N)
    X = mu[comp] + rng.standard_normal((N, d))
    W, b, groups = make_nodes(rng, d, L, int(round(dup_frac * L)))
    return Problem("mixture_rankdef", X, W, b, one_hot(comp, m), comp.astype(np.int64), groups)


def smooth_regression(seed: int = 4, N: int = 500000, L: int = 10000, d: int = 128, m: int = 4,
                      n_terms: int = 32, noise_sd: float = 0.1) -> Problem:
    """Precision-form regression: X ~ N(0, I_d) rows, L distinct nodes (full
    rank), m outputs t_k(x) = sum_j a_jk cos(omega_j . x + phi_j) + noise with
    omega_j ~ N(0, I/d), phi_j ~ U[0, 2pi), a_jk ~ N(0, 1/n_terms) and noise of
    variance 0.01 (standard deviation 0.1)."""
    rng = np.random.default_rng(seed)
    X = rng.standard_normal((N, d))
    W, b, groups = make_nodes(rng, d, L, 0)
    omega = rng.standard_normal((d, n_terms)) / math.sqrt(d)
    phi = rng.uniform(0.0, 2.0 * math.pi, size=n_terms)
    a = rng.standard_normal((n_terms, m)) / math.sqrt(n_terms)
    T = np.empty((N, m))
    for s in range(0, N, 65536):
        T[s:s + 65536] = np.cos(X[s:s + 65536] @ omega + phi) @ a
    T += noise_sd * rng.standard_normal((N, m))
    return Problem("smooth_regression", X, W, b, T, None, groups)


def batch_sweep(seed: int = 5, count: int = 256, d: int = 32, m: int = 5,
                L_range=(64, 2048), N_range=(1000, 50000), dup_frac: float = 0.1) -> List[Problem]:
    """Hidden-size sweep: `count` independent ELMs with L and N drawn
    log-uniform, d=32 features U[-1,1], 5 one-hot classes by argmax of a random
    linear map, 10% duplicated nodes in each ELM.  Per-ELM streams are spawned
    from the master seed so each ELM is reproducible on its own."""
    ss = np.random.SeedSequence(seed)
    top = np.random.default_rng(ss)
    Ls = np.rint(np.exp(top.uniform(math.log(L_range[0]), math.log(L_range[1]), size=count))).astype(int)
    Ns = np.rint(np.exp(top.uniform(math.log(N_range[0]), math.log(N_range[1]), size=count))).astype(int)
    out = []
    for e, child in enumerate(ss.spawn(count)):
        rng = np.random.default_rng(child)
        N, L = int(Ns[e]), int(Ls[e])
        X = rng.uniform(-1.0, 1.0, size=(N, d))
        W, b, groups = make_nodes(rng, d, L, int(round(dup_frac * L)))
        V = rng.standard_normal((d, m))
        labels = np.argmax(X @ V, axis=1).astype(np.int64)
        out.append(Problem(f"batch_sweep[{e}]", X, W, b, one_hot(labels, m), labels, groups))
    return out


def gina_shape(L: int, seed: int = 7) -> Problem:
    """Shape of the paper's GINA runs (Table 1): N=3468, d=971, given L; two
    one-hot classes from a random linear rule.  Context only (the dataset
    itself is not available)."""
    rng = np.random.default_rng(seed)
    N, d = 3468, 971
    X = rng.uniform(0.0, 1.0, size=(N, d)) * (rng.uniform(0.0, 1.0, size=(N, d)) < 0.2)
    W, b, groups = make_nodes(rng, d, L, 0)
    v = rng.standard_normal(d)
    labels = (X @ v > np.median(X @ v)).astype(np.int64)
    return Problem(f"gina_shape_L{L}", X, W, b, one_hot(labels, 2), labels, groups)


def random_problem(seed: int, N: int, d: int, L: int, m: int, n_dup: int = 0,
                   x_low: float = -1.0, x_high: float = 1.0) -> Problem:
    """Small generic problem for parity sweeps (ragged sizes, N<L, ...)."""
    rng = np.random.default_rng(seed)
    X = rng.uniform(x_low, x_high, size=(N, d))
    W, b, groups = make_nodes(rng, d, L, n_dup)
    labels = rng.integers(0, m, size=N)
    return Problem(f"random[{seed},{N},{d},{L},{m},{n_dup}]", X, W, b, one_hot(labels, m), labels, groups)


WORKLOADS = {
    "tiny_fp64": tiny_fp64,
    "digits_like": digits_like,
    "mixture_rankdef": mixture_rankdef,
    "smooth_regression": smooth_regression,
}
