"""Seeded synthetic workloads for parallel brute-force Bayesian cross-validation.

This module only *generates inputs*: design matrices, responses, fold
specifications, sampler settings and initial chain positions.  It holds none of
the method's arithmetic (no log densities, no gradients, no HMC, no
accumulators).  Both the CPU oracle and the HIP library consume what it makes,
and neither imports the other.

The paper's real datasets (rats, radon, air passengers; Section 5) are not
available, so five synthetic configurations shaped like its workloads stand in
for them:

  c1  LOO-CV, conjugate Gaussian linear regression (n=100, p=5, K=100, L=4)
  c2  LOGO-CV, hierarchical logistic regression (50 groups of 20..200 rows,
      p=10, K=50, L=16)  -- grouped data as in Example 1 / the radon example
  c3  hv-block CV of a Gaussian AR(4) series (T=5000, v=5, h=10, K=1000, L=8)
      -- time-series blocked CV as in the air-passenger example
  c4  K-fold CV of a Poisson log-link GLM (n=20000, p=64, K=500, L=8)
  c5  blocked CV of a logistic GLM (n=100000, p=128, K=10000, L=4)
  ex1 the paper's Example 1: LOGO-CV of a grouped Gaussian regression with
      hierarchical intercepts and unknown noise scale (J=50 groups of 5 rows,
      4 group-level covariates, K=50, L=4), model A (all covariates) against
      model B (one dropped)

Settings the paper leaves open (step size, mass matrix, warm-up length, the
full-data fit that seeds the chains) are fixed here; the reasoning for each is
recorded with the design notes of the repository.

Step 1 of the workflow (full-data inference, Section 3) is replaced by a
stand-in computed from the data-generating process: the inverse mass matrix is
the diagonal of (prior precision + Fisher information at the true parameter)^-1
and chains start at the true parameter plus Gaussian noise of that scale.
"""
from __future__ import annotations

import dataclasses
import math
from typing import Optional

import numpy as np

# Likelihood families (same numbering as the C header).
GAUSSIAN = 0
LOGISTIC = 1
POISSON = 2
HIER_LOGISTIC = 3
HIER_GAUSSIAN = 4
HIER_FAMILIES = (HIER_LOGISTIC, HIER_GAUSSIAN)

# Arithmetic used by the GPU path for the contractions.
PREC_FP64 = 0
PREC_FP32 = 1
PREC_BF16X3 = 2
PREC_BF16X5 = 3
PREC_FP64_UNFUSED = 4

# Fold encodings.
FOLDS_INDEX = 0
FOLDS_INTERVALS = 1
FOLDS_DENSE = 2

ROLE_EXCLUDED = 0
ROLE_TRAIN = 1
ROLE_TEST = 2

DATA_SEED_BASE = 20231007 * 10


@dataclasses.dataclass
class Workload:
    name: str
    family: int
    precision: int
    X: np.ndarray              # [n, p] float64 (for bf16 workloads exactly hi+lo)
    y: np.ndarray              # [n] float64
    K: int
    L: int
    fold_kind: int
    fold_index: Optional[np.ndarray] = None   # [n] int32 (INDEX)
    intervals: Optional[np.ndarray] = None    # [K, 4] int64 (INTERVALS)
    roles: Optional[np.ndarray] = None        # [K, n] int8 (DENSE)
    group_of: Optional[np.ndarray] = None     # [n] int32 (hierarchical families)
    n_groups: int = 0
    sigma: float = 1.0
    prior_scale: Optional[np.ndarray] = None  # [d]
    step_size: float = 0.1
    n_leapfrog: int = 8
    inv_mass: Optional[np.ndarray] = None     # [d]
    init_pos: Optional[np.ndarray] = None     # [C, d]
    n_warmup: int = 250
    n_samples: int = 1000
    batch_size: int = 50
    n_blocks: int = 5
    seed: int = 0                              # Philox key of the sampler
    chain_offset: int = 0                      # global id of chain 0
    rhat_mode: int = 0                         # 0 Welford blocks, 1 shifted sums (Algorithm A2)
    scores: int = 0                            # extra scores accumulated: 1 HS, 2 DSS (bit mask)
    store_draws: int = 0                       # post-warm-up draws of s kept on the device (Algorithm 1)
    n_models: int = 1                          # nested models in one launch (Appendix B)
    model_mask: Optional[np.ndarray] = None    # [n_models, p] uint8: covariate j used by model m
    truth: Optional[np.ndarray] = None         # [d]
    x_hi: Optional[np.ndarray] = None          # [n, p] uint16 bf16 bits
    x_lo: Optional[np.ndarray] = None          # [n, p] uint16 bf16 bits

    @property
    def n(self) -> int:
        return int(self.X.shape[0])

    @property
    def p(self) -> int:
        return int(self.X.shape[1])

    @property
    def d(self) -> int:
        if self.family == HIER_LOGISTIC:
            return self.p + 2 + self.n_groups
        if self.family == HIER_GAUSSIAN:
            return self.p + 3 + self.n_groups
        return self.p

    @property
    def C(self) -> int:
        return self.n_models * self.K * self.L

    @property
    def batches_per_block(self) -> int:
        return max(1, self.n_samples // (self.batch_size * self.n_blocks))

    @property
    def n_iter(self) -> int:
        return self.n_warmup + self.n_samples


# ----------------------------------------------------------------------------
# bf16 helpers (data format only): round-to-nearest-even float32 -> bf16 bits
# ----------------------------------------------------------------------------

def _bf16_bits_rne(x32: np.ndarray) -> np.ndarray:
    u = np.ascontiguousarray(x32, dtype=np.float32).view(np.uint32).astype(np.uint64)
    lsb = (u >> np.uint64(16)) & np.uint64(1)
    u = (u + np.uint64(0x7FFF) + lsb) & np.uint64(0xFFFF0000)
    return (u >> np.uint64(16)).astype(np.uint16)


def bf16_bits_to_f64(b: np.ndarray) -> np.ndarray:
    u = b.astype(np.uint32) << np.uint32(16)
    return u.view(np.float32).astype(np.float64)


def split_hi_lo(x32: np.ndarray):
    """Two bf16 planes (hi, lo) whose exact sum is the stored design matrix."""
    hi = _bf16_bits_rne(x32)
    rem = (x32.astype(np.float32) - bf16_bits_to_f64(hi).astype(np.float32)).astype(np.float32)
    lo = _bf16_bits_rne(rem)
    return hi, lo


# ----------------------------------------------------------------------------
# Step-1 stand-in: tuning from the data-generating process
# ----------------------------------------------------------------------------

def _glm_link_weight(family: int, eta: np.ndarray, sigma: float) -> np.ndarray:
    """Fisher weight of one observation at linear predictor eta (DGP moment)."""
    if family == GAUSSIAN:
        return np.full_like(eta, 1.0 / sigma ** 2)
    if family in (LOGISTIC, HIER_LOGISTIC):
        pr = 1.0 / (1.0 + np.exp(-eta))
        return pr * (1.0 - pr)
    if family == POISSON:
        return np.exp(eta)
    raise ValueError(family)


def _diag_cov_from_precision(P: np.ndarray) -> np.ndarray:
    return np.diag(np.linalg.inv(P)).copy()


def _init_positions(rng: np.random.Generator, center: np.ndarray, inv_mass: np.ndarray,
                    C: int) -> np.ndarray:
    z = rng.standard_normal((C, center.shape[0]))
    return center[None, :] + np.sqrt(inv_mass)[None, :] * z


# ----------------------------------------------------------------------------
# The five configurations
# ----------------------------------------------------------------------------

def make_c1(seed_offset: int = 1) -> Workload:
    """LOO-CV of conjugate Gaussian regression, n=100, p=5, sigma=0.5 known."""
    seed = DATA_SEED_BASE + seed_offset
    rng = np.random.default_rng(seed)
    n, p, sigma = 100, 5, 0.5
    X = rng.standard_normal((n, p))
    beta = rng.standard_normal(p)
    y = X @ beta + sigma * rng.standard_normal(n)
    K, L = n, 4
    prior_scale = np.ones(p)
    # Exact full-data posterior covariance (conjugate) -> diagonal inverse mass.
    prec = np.eye(p) + X.T @ X / sigma ** 2
    inv_mass = _diag_cov_from_precision(prec)
    init = _init_positions(np.random.default_rng([seed, 1]), beta, inv_mass, K * L)
    return Workload(
        name="c1_loo_gaussian", family=GAUSSIAN, precision=PREC_FP64, X=X, y=y, K=K, L=L,
        fold_kind=FOLDS_INDEX, fold_index=np.arange(n, dtype=np.int32), sigma=sigma,
        prior_scale=prior_scale, step_size=0.1, n_leapfrog=8, inv_mass=inv_mass,
        init_pos=init, n_warmup=250, n_samples=1000, batch_size=50, n_blocks=5,
        seed=seed + 1, truth=beta)


def make_c2(seed_offset: int = 2) -> Workload:
    """LOGO-CV of a non-centred hierarchical logistic regression.

    theta = [beta (p), mu, u = log tau, z (G)];  eta = x'beta + mu + exp(u) z_g.
    """
    seed = DATA_SEED_BASE + seed_offset
    rng = np.random.default_rng(seed)
    G, p = 50, 10
    sizes = rng.integers(20, 201, size=G)
    group_of = np.repeat(np.arange(G, dtype=np.int32), sizes)
    n = int(sizes.sum())
    X = rng.standard_normal((n, p))
    beta = rng.standard_normal(p)
    mu = rng.standard_normal()
    tau = abs(rng.standard_normal())
    z = rng.standard_normal(G)
    eta = X @ beta + mu + tau * z[group_of]
    y = (rng.random(n) < 1.0 / (1.0 + np.exp(-eta))).astype(np.float64)
    d = p + 2 + G
    truth = np.concatenate([beta, [mu, math.log(tau)], z])
    # Fisher information at the truth for theta (Jacobian of eta wrt theta).
    w = _glm_link_weight(LOGISTIC, eta, 1.0)
    J = np.zeros((n, d))
    J[:, :p] = X
    J[:, p] = 1.0
    J[:, p + 1] = tau * z[group_of]
    J[np.arange(n), p + 2 + group_of] = tau
    prec = J.T @ (w[:, None] * J)
    prior_prec = np.ones(d)
    prior_prec[p + 1] = 2.0 * tau ** 2          # -d2/du2 of the log-half-normal + Jacobian
    prec[np.diag_indices(d)] += prior_prec
    inv_mass = _diag_cov_from_precision(prec)
    K, L = G, 16
    init = _init_positions(np.random.default_rng([seed, 1]), truth, inv_mass, K * L)
    prior_scale = np.ones(d)
    return Workload(
        name="c2_logo_hier_logistic", family=HIER_LOGISTIC, precision=PREC_FP32, X=X, y=y,
        K=K, L=L, fold_kind=FOLDS_INDEX, fold_index=group_of.copy(), group_of=group_of,
        n_groups=G, prior_scale=prior_scale, step_size=0.25, n_leapfrog=8,
        inv_mass=inv_mass, init_pos=init, n_warmup=250, n_samples=1000, batch_size=50,
        n_blocks=5, seed=seed + 1, truth=truth)


EX1_SCALE_VAR = 10.0    # variance of N(0, 10) designs and of the half-normal scale priors


def make_ex1(seed_offset: int = 6, J: int = 50, Nj: int = 5) -> Workload:
    """Example 1 (Section 2): grouped Gaussian regression, LOGO-CV.

    J = 50 groups of N_j = 5 rows; the J x 4 group-level design has N(0, 10)
    entries and row i of group j carries x_j.  True values are drawn from the
    priors: beta ~ N(0, I), mu ~ N(0, 1), sigma_a and sigma_y half-normal with
    variance 10, alpha_j ~ N(mu, sigma_a^2); y_ij ~ N(alpha_j + x_j'beta,
    sigma_y^2).  theta = [beta (4), mu, log sigma_a, log sigma_y, z (J)] with
    alpha_j = mu + sigma_a z_j.  K = J folds, L = 4 chains.  (J and Nj other
    than 50 and 5 give larger instances of the same model.)
    """
    seed = DATA_SEED_BASE + seed_offset
    rng = np.random.default_rng(seed)
    p = 4
    sd = math.sqrt(EX1_SCALE_VAR)
    Xg = sd * rng.standard_normal((J, p))
    group_of = np.repeat(np.arange(J, dtype=np.int32), Nj)
    X = Xg[group_of].copy()
    n = X.shape[0]
    beta = rng.standard_normal(p)
    mu = rng.standard_normal()
    sig_a = abs(sd * rng.standard_normal())
    sig_y = abs(sd * rng.standard_normal())
    z = rng.standard_normal(J)
    eta = X @ beta + mu + sig_a * z[group_of]
    y = eta + sig_y * rng.standard_normal(n)
    d = p + 3 + J
    truth = np.concatenate([beta, [mu, math.log(sig_a), math.log(sig_y)], z])
    # Fisher information at the truth (Jacobian of eta wrt theta, Gaussian
    # weight 1/sigma_y^2; log sigma_y: 2 per row) plus the prior curvature
    Jm = np.zeros((n, d))
    Jm[:, :p] = X
    Jm[:, p] = 1.0
    Jm[:, p + 1] = sig_a * z[group_of]
    Jm[np.arange(n), p + 3 + group_of] = sig_a
    prec = Jm.T @ Jm / sig_y ** 2
    prec[p + 2, p + 2] = 2.0 * n
    prior_prec = np.ones(d)
    prior_prec[p + 1] = 2.0 * sig_a ** 2 / EX1_SCALE_VAR
    prior_prec[p + 2] = 2.0 * sig_y ** 2 / EX1_SCALE_VAR
    prec[np.diag_indices(d)] += prior_prec
    inv_mass = _diag_cov_from_precision(prec)
    K, L = J, 4
    init = _init_positions(np.random.default_rng([seed, 1]), truth, inv_mass, K * L)
    return Workload(
        name="ex1_logo_hier_gaussian", family=HIER_GAUSSIAN, precision=PREC_FP64, X=X, y=y,
        K=K, L=L, fold_kind=FOLDS_INDEX, fold_index=group_of.copy(), group_of=group_of,
        n_groups=J, prior_scale=np.ones(d), step_size=0.25, n_leapfrog=8,
        inv_mass=inv_mass, init_pos=init, n_warmup=250, n_samples=1000, batch_size=50,
        n_blocks=5, seed=seed + 1, truth=truth)


def make_ex1_ab(seed_offset: int = 6) -> Workload:
    """Example 1's two models in one launch (Sections 2 and 2.3): model A
    uses all 4 covariates, model B drops one, the covariate whose true
    coefficient is largest in magnitude (the paper does not say which)."""
    w = make_ex1(seed_offset)
    masks = np.ones((2, w.p), dtype=np.uint8)
    masks[1, int(np.argmax(np.abs(w.truth[:w.p])))] = 0
    return with_models(w, masks)


AR4_RHO = np.array([0.86, -0.5016, 0.284, -0.1])


def make_c3(seed_offset: int = 3) -> Workload:
    """hv-block CV of a Gaussian AR(4) series (sigma=1 known), conditional likelihood."""
    seed = DATA_SEED_BASE + seed_offset
    rng = np.random.default_rng(seed)
    T, burn, lags = 5000, 500, 4
    e = rng.standard_normal(T + burn)
    series = np.zeros(T + burn)
    for t in range(T + burn):
        acc = e[t]
        for j in range(lags):
            if t - 1 - j >= 0:
                acc += AR4_RHO[j] * series[t - 1 - j]
        series[t] = acc
    s = series[burn:]                       # y_1 .. y_T  (index 0 .. T-1)
    rows = np.arange(lags, T)               # t = 5 .. 5000 in 1-based terms
    X = np.stack([s[rows - 1 - j] for j in range(lags)], axis=1)
    y = s[rows].copy()
    n = X.shape[0]                          # 4996
    v, h, stride = 5, 10, 5
    K = (n + stride - 1) // stride          # 1000 (last block holds one row)
    iv = np.zeros((K, 4), dtype=np.int64)
    for k in range(K):
        lo = k * stride
        hi = min(lo + v, n)
        iv[k] = (lo, hi, max(0, lo - h), min(n, hi + h))
    sigma = 1.0
    prec = np.eye(lags) + X.T @ X / sigma ** 2
    inv_mass = _diag_cov_from_precision(prec)
    L = 8
    init = _init_positions(np.random.default_rng([seed, 1]), AR4_RHO.copy(), inv_mass, K * L)
    return Workload(
        name="c3_hvblock_ar4", family=GAUSSIAN, precision=PREC_FP64, X=X, y=y, K=K, L=L,
        fold_kind=FOLDS_INTERVALS, intervals=iv, sigma=sigma, prior_scale=np.ones(lags),
        step_size=0.1, n_leapfrog=8, inv_mass=inv_mass, init_pos=init, n_warmup=250,
        n_samples=1000, batch_size=50, n_blocks=5, seed=seed + 1, truth=AR4_RHO.copy())


def _bf16_design(rng: np.random.Generator, n: int, p: int):
    x32 = (rng.standard_normal((n, p)) / math.sqrt(p)).astype(np.float32)
    hi, lo = split_hi_lo(x32)
    X = bf16_bits_to_f64(hi) + bf16_bits_to_f64(lo)
    return X, hi, lo


def make_c4(seed_offset: int = 4) -> Workload:
    """K-fold CV (500 folds x 40 rows) of a Poisson log-link GLM, n=20000, p=64."""
    seed = DATA_SEED_BASE + seed_offset
    rng = np.random.default_rng(seed)
    n, p, K, L = 20000, 64, 500, 8
    X, hi, lo = _bf16_design(rng, n, p)
    beta = 0.3 * rng.standard_normal(p)
    eta = X @ beta
    y = rng.poisson(np.exp(eta)).astype(np.float64)
    perm = rng.permutation(n)
    fold_index = np.empty(n, dtype=np.int32)
    fold_index[perm] = (np.arange(n) // (n // K)).astype(np.int32)
    prior_scale = np.full(p, 0.3)
    w = _glm_link_weight(POISSON, eta, 1.0)
    prec = X.T @ (w[:, None] * X) + np.diag(1.0 / prior_scale ** 2)
    inv_mass = _diag_cov_from_precision(prec)
    init = _init_positions(np.random.default_rng([seed, 1]), beta, inv_mass, K * L)
    return Workload(
        name="c4_kfold_poisson", family=POISSON, precision=PREC_BF16X3, X=X, y=y, K=K, L=L,
        fold_kind=FOLDS_INDEX, fold_index=fold_index, prior_scale=prior_scale,
        step_size=0.2, n_leapfrog=8, inv_mass=inv_mass, init_pos=init, n_warmup=250,
        n_samples=1000, batch_size=50, n_blocks=5, seed=seed + 1, truth=beta,
        x_hi=hi, x_lo=lo)


def make_c5(seed_offset: int = 5) -> Workload:
    """Blocked CV (10000 contiguous 10-row blocks) of a logistic GLM, n=1e5, p=128."""
    seed = DATA_SEED_BASE + seed_offset
    rng = np.random.default_rng(seed)
    n, p, block, L = 100000, 128, 10, 4
    K = n // block
    X, hi, lo = _bf16_design(rng, n, p)
    beta = rng.standard_normal(p)
    eta = X @ beta
    y = (rng.random(n) < 1.0 / (1.0 + np.exp(-eta))).astype(np.float64)
    block_fold = rng.permutation(K).astype(np.int32)
    fold_index = np.repeat(block_fold, block).astype(np.int32)
    prior_scale = np.ones(p)
    w = _glm_link_weight(LOGISTIC, eta, 1.0)
    prec = X.T @ (w[:, None] * X) + np.eye(p)
    inv_mass = _diag_cov_from_precision(prec)
    init = _init_positions(np.random.default_rng([seed, 1]), beta, inv_mass, K * L)
    return Workload(
        name="c5_blocked_logistic", family=LOGISTIC, precision=PREC_BF16X3, X=X, y=y, K=K,
        L=L, fold_kind=FOLDS_INDEX, fold_index=fold_index, prior_scale=prior_scale,
        step_size=0.2, n_leapfrog=8, inv_mass=inv_mass, init_pos=init, n_warmup=500,
        n_samples=2000, batch_size=50, n_blocks=5, seed=seed + 1, truth=beta,
        x_hi=hi, x_lo=lo)


MAKERS = {"c1": make_c1, "c2": make_c2, "c3": make_c3, "c4": make_c4, "c5": make_c5, "ex1": make_ex1,
          "ex1_ab": lambda: make_ex1_ab()}


def make(name: str) -> Workload:
    return MAKERS[name]()


# ----------------------------------------------------------------------------
# Fold subsets: the same chains (same global chain ids, hence the same random
# streams) restricted to a contiguous range of folds.
# ----------------------------------------------------------------------------

def fold_subset(w: Workload, k0: int, k1: int) -> Workload:
    assert 0 <= k0 < k1 <= w.K
    sub = dataclasses.replace(w)
    sub.K = k1 - k0
    sub.chain_offset = w.chain_offset + k0 * w.L
    sub.init_pos = w.init_pos[k0 * w.L:k1 * w.L].copy()
    if w.fold_kind == FOLDS_INDEX:
        fi = w.fold_index.astype(np.int64)
        inside = (fi >= k0) & (fi < k1)
        sub.fold_index = np.where(inside, fi - k0, -1).astype(np.int32)
    elif w.fold_kind == FOLDS_INTERVALS:
        sub.intervals = w.intervals[k0:k1].copy()
    else:
        sub.roles = w.roles[k0:k1].copy()
    return sub


def full_data(w: Workload, L: int = 8, n_warmup: int = 1000) -> Workload:
    """The full-data model of w (the workflow's Step 1): one fold whose rows
    all train (fold id -1 everywhere, so no held-out rows and s = 0), L
    chains started at the first L of w's starting positions, a unit inverse
    mass and w's step size as the adaptation's starting point, and n_warmup
    transitions counted as warm-up (no accumulation during adaptation)."""
    sub = dataclasses.replace(w)
    sub.name = w.name + "_full"
    sub.K, sub.L = 1, L
    sub.fold_kind = FOLDS_INDEX
    sub.fold_index = np.full(w.n, -1, dtype=np.int32)
    sub.intervals = None
    sub.roles = None
    sub.chain_offset = 0
    sub.init_pos = np.array(w.init_pos[:L], dtype=np.float64)
    sub.inv_mass = np.ones(w.d)
    sub.n_warmup = n_warmup
    sub.scores = 0
    sub.store_draws = 0
    return sub


def with_models(w: Workload, masks) -> Workload:
    """Several nested GLMs of w in one launch (Appendix B, parallel model
    evaluation): masks [M, p] of 0/1, model m uses covariate j iff
    masks[m, j].  Chains are model-major (M x K x L); every model's chains
    start where w's do and use its random streams shifted by K*L per model
    (global chain ids)."""
    masks = np.ascontiguousarray(np.atleast_2d(masks), dtype=np.uint8)
    assert masks.shape[1] == w.p and w.family != HIER_LOGISTIC and w.n_models == 1
    sub = dataclasses.replace(w)
    sub.name = w.name + f"_{masks.shape[0]}models"
    sub.n_models = masks.shape[0]
    sub.model_mask = masks
    sub.init_pos = np.concatenate([w.init_pos] * masks.shape[0], axis=0)
    return sub


def model_of(w: Workload, m: int) -> Workload:
    """Model m of a multi-model workload as a workload of its own: the masked
    covariates' columns zeroed (the masked form of Appendix B) and its global
    chain ids, so the oracle can replay its chains."""
    cols = np.flatnonzero(w.model_mask[m] == 0)
    base = dataclasses.replace(w, n_models=1, model_mask=None)
    sub = drop_covariates(base, cols, zero=True) if cols.size else dataclasses.replace(base)
    sub.chain_offset = w.chain_offset + m * w.K * w.L
    sub.init_pos = w.init_pos[m * w.K * w.L:(m + 1) * w.K * w.L].copy()
    return sub


def drop_covariates(w: Workload, cols, zero: bool = False) -> Workload:
    """The same workload for the model without covariates `cols` (GLM
    families): the nested-model comparison of Section 2.3, model B missing
    covariates of model A.  Same folds, rows and random streams; the prior
    scales, mass-matrix entries and initial positions of the kept covariates
    are those of the full model.  zero=True keeps p and zeroes the columns
    instead (the masked form of Appendix B: the dropped coefficients remain
    as parameters the likelihood ignores), for paths built for fixed p; that
    form also serves the hierarchical Gaussian family."""
    assert w.family in (GAUSSIAN, LOGISTIC, POISSON) or (zero and w.family == HIER_GAUSSIAN), \
        "GLM families (and the hierarchical Gaussian with zero=True) only"
    if zero:
        sub = dataclasses.replace(w)
        sub.name = w.name + "_zero_" + "_".join(str(int(c)) for c in np.atleast_1d(cols))
        sub.X = w.X.copy()
        sub.X[:, cols] = 0.0
        if w.x_hi is not None:
            sub.x_hi = w.x_hi.copy()
            sub.x_lo = w.x_lo.copy()
            sub.x_hi[:, cols] = 0
            sub.x_lo[:, cols] = 0
        return sub
    keep = np.setdiff1d(np.arange(w.p), np.asarray(cols))
    sub = dataclasses.replace(w)
    sub.name = w.name + "_minus_" + "_".join(str(int(c)) for c in np.atleast_1d(cols))
    sub.X = np.ascontiguousarray(w.X[:, keep])
    if w.x_hi is not None:
        sub.x_hi = np.ascontiguousarray(w.x_hi[:, keep])
        sub.x_lo = np.ascontiguousarray(w.x_lo[:, keep])
    sub.prior_scale = None if w.prior_scale is None else w.prior_scale[keep].copy()
    sub.inv_mass = w.inv_mass[keep].copy()
    sub.init_pos = np.ascontiguousarray(w.init_pos[:, keep])
    sub.truth = None if w.truth is None else np.asarray(w.truth)[keep].copy()
    return sub


def with_dense_roles(w: Workload) -> Workload:
    """Same workload with its folds given as a dense K x n role matrix."""
    roles = np.full((w.K, w.n), ROLE_TRAIN, dtype=np.int8)
    if w.fold_kind == FOLDS_INDEX:
        for k in range(w.K):
            roles[k, w.fold_index == k] = ROLE_TEST
    elif w.fold_kind == FOLDS_INTERVALS:
        for k, (lo, hi, elo, ehi) in enumerate(w.intervals):
            roles[k, elo:ehi] = ROLE_EXCLUDED
            roles[k, lo:hi] = ROLE_TEST
    else:
        roles = w.roles.copy()
    sub = dataclasses.replace(w)
    sub.fold_kind = FOLDS_DENSE
    sub.roles = roles
    sub.fold_index = None
    sub.intervals = None
    return sub
