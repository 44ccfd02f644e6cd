"""Seeded synthetic inputs for the latent-GP RMHMC workloads.

This module only *draws inputs*: covariates, labels and the hyperparameter
layout of each model.  It holds
none of the sampler's arithmetic (no Hessian, metric, integrator or chain
code).  The one piece of kernel arithmetic here is the GP prior draw of the
synthetic ground-truth function, which is part of the data recipe: the
Gram matrix is written out directly below for that purpose only.

Both the GPU path and the FP64 reference use these generators, so the two
always see bit-identical inputs.

Model conventions (the paper's experiments use a reduced-rank basis model;
these workloads sample the latent GP values f at the N inputs instead, the
parameterisation the paper's Discussion attributes to earlier work):

* q = (f_1..f_N, eta_1..eta_P); f first, then the log-hyperparameters.
* K(eta) = sum of kernel terms + jitter * I (jitter fixed, not sampled).
* Kernel terms (parameters are consumed in term order):
    SE_ISO(cols):      s^2 exp(-|x-x'|^2 / (2 l^2)),    eta = (log s, log l)
    SE_ARD(cols):      s^2 exp(-sum_d r_d^2/(2 l_d^2)), eta = (log s, log l_d...)
    LINEAR_ARD(cols):  sum_d v_d x_d x'_d,              eta = (log v_d...)
    BINARY_SAME(col):  s^2 [x_c == x'_c],               eta = (log s,)
* Priors: eta ~ N(0, I); f | eta ~ N(0, K(eta)).
* Likelihood: Bernoulli-logit (y in {0,1}) scaled by an inverse temperature
  beta (power posterior), Gaussian with known noise variance (tests), or the
  mean/variance model of Sec. 2.1 Example 1 (J = 2 latent functions).
* Several latent functions (J = 2): the latent points are stacked, function
  by function (f_1 at the R records, then f_2 at the same records); the
  column fn_col of X holds each point's function index, and a kernel term
  with term_fns[t] = j acts only between two points of function j, so K is
  block diagonal, one block per function with its own hyperparameters.
"""
from __future__ import annotations

import dataclasses
import math
from typing import List, Sequence, Tuple

import numpy as np

SE_ISO = 0
SE_ARD = 1
LINEAR_ARD = 2
BINARY_SAME = 3

LIK_BERNOULLI_LOGIT = 0
LIK_GAUSSIAN = 1
LIK_GAUSSIAN_MV = 2     # Example 1 of Sec. 2.1: mean f_1, variance delta + exp(f_2)

KIND_NAMES = {SE_ISO: "se_iso", SE_ARD: "se_ard", LINEAR_ARD: "linear_ard",
              BINARY_SAME: "binary_same"}


def term_nparams(kind: int, cols: Sequence[int]) -> int:
    if kind == SE_ISO:
        return 2
    if kind == SE_ARD:
        return 1 + len(cols)
    if kind == LINEAR_ARD:
        return len(cols)
    if kind == BINARY_SAME:
        if len(cols) != 1:
            raise ValueError("BINARY_SAME takes exactly one column")
        return 1
    raise ValueError(f"unknown kernel kind {kind}")


@dataclasses.dataclass
class ModelSpec:
    """Plain description of one latent-GP model (host arrays, FP64)."""
    X: np.ndarray                     # N x dx covariates
    y: np.ndarray                     # N labels ({0,1}) or targets (Gaussian)
    terms: List[Tuple[int, Tuple[int, ...]]]
    lik: int = LIK_BERNOULLI_LOGIT
    noise_var: float = 1.0            # Gaussian likelihood only
    jitter: float = 1e-6
    beta: float = 1.0                 # inverse temperature on the likelihood
    delta: float = 0.0                # variance floor of the mean/variance model
    fn_col: int = -1                # column of X with each point's function index
    term_fns: Tuple[int, ...] = ()  # function index of each term (-1: all points)

    def __post_init__(self):
        self.X = np.ascontiguousarray(np.asarray(self.X, dtype=np.float64))
        if self.X.ndim != 2:
            raise ValueError("X must be N x dx")
        self.y = np.ascontiguousarray(np.asarray(self.y, dtype=np.float64))
        self.terms = [(int(k), tuple(int(c) for c in cols)) for k, cols in self.terms]
        for k, cols in self.terms:
            term_nparams(k, cols)
            for c in cols:
                if not 0 <= c < self.X.shape[1]:
                    raise ValueError("kernel column out of range")
        self.term_fns = tuple(int(t) for t in self.term_fns)
        if self.term_fns and len(self.term_fns) != len(self.terms):
            raise ValueError("term_fns needs one entry per kernel term")
        if self.term_fns and not 0 <= self.fn_col < self.X.shape[1]:
            raise ValueError("term_fns needs a task column")
        if self.lik == LIK_GAUSSIAN_MV:
            if self.X.shape[0] % 2 or self.delta <= 0.0 or self.fn_col < 0:
                raise ValueError("the mean/variance model needs 2R stacked points, delta > 0 "
                                 "and a task column")

    @property
    def N(self) -> int:
        return self.X.shape[0]

    @property
    def dx(self) -> int:
        return self.X.shape[1]

    @property
    def n_records(self) -> int:
        """Data records: N, or N / 2 for the two stacked latent functions."""
        return self.N // 2 if self.lik == LIK_GAUSSIAN_MV else self.N

    @property
    def P(self) -> int:
        return sum(term_nparams(k, c) for k, c in self.terms)

    @property
    def D(self) -> int:
        return self.N + self.P


def _gram_for_data(X, terms, eta, jitter):
    """Kernel Gram matrix used only to draw the synthetic ground truth."""
    N = X.shape[0]
    K = np.zeros((N, N))
    i = 0
    for kind, cols in terms:
        if kind in (SE_ISO, SE_ARD):
            s = math.exp(eta[i])
            r2 = np.zeros((N, N))
            for j, c in enumerate(cols):
                ell = math.exp(eta[i + 1] if kind == SE_ISO else eta[i + 1 + j])
                r2 += (X[:, c, None] - X[None, :, c]) ** 2 / ell ** 2
            K += s * s * np.exp(-0.5 * r2)
        elif kind == LINEAR_ARD:
            for j, c in enumerate(cols):
                K += math.exp(eta[i + j]) * np.outer(X[:, c], X[:, c])
        elif kind == BINARY_SAME:
            c = cols[0]
            K += math.exp(2 * eta[i]) * (X[:, c, None] == X[None, :, c])
        i += term_nparams(kind, cols)
    return K + jitter * np.eye(N)


def _finish(rng, X, terms, jitter=1e-6, beta=1.0):
    """Draw eta_true ~ N(0, I), f_true ~ GP, labels ~ Bernoulli(sigmoid(f))."""
    P = sum(term_nparams(k, c) for k, c in terms)
    eta_true = rng.standard_normal(P)
    L = np.linalg.cholesky(_gram_for_data(X, terms, eta_true, jitter))
    f_true = L @ rng.standard_normal(X.shape[0])
    y = (rng.uniform(size=X.shape[0]) < 1.0 / (1.0 + np.exp(-f_true))).astype(np.float64)
    spec = ModelSpec(X=X, y=y, terms=list(terms), jitter=jitter, beta=beta)
    return spec, eta_true, f_true


def gp_logistic_2d(N: int, seed: int = 0, beta: float = 1.0):
    """GP classification on 2-D inputs x ~ U[-1,1]^2 with an isotropic SE kernel."""
    rng = np.random.default_rng(seed)
    X = rng.uniform(-1.0, 1.0, size=(N, 2))
    return _finish(rng, X, [(SE_ISO, (0, 1))], beta=beta)


def gp_logistic_ard4(N: int = 256, seed: int = 0):
    """GP classification on 4-D inputs x ~ N(0, I) with an SE-ARD kernel."""
    rng = np.random.default_rng(seed)
    X = rng.standard_normal((N, 4))
    return _finish(rng, X, [(SE_ARD, (0, 1, 2, 3))])


def propensity_mkl(N: int = 1024, seed: int = 0):
    """Binary-treatment propensity model with a multiple-kernel sum.

    8 covariates: 5 continuous N(0,1) and 3 binary Bernoulli(0.3).  Kernel =
    SE-ARD(5 continuous) + linear-ARD(5 continuous) + one same-value kernel per
    binary covariate: 6 + 5 + 3 = 14 hyperparameters.  Synthetic stand-in for
    the shape of the paper's medical-expenditure propensity analysis.
    """
    rng = np.random.default_rng(seed)
    Xc = rng.standard_normal((N, 5))
    Xb = (rng.uniform(size=(N, 3)) < 0.3).astype(np.float64)
    X = np.concatenate([Xc, Xb], axis=1)
    terms = [(SE_ARD, (0, 1, 2, 3, 4)), (LINEAR_ARD, (0, 1, 2, 3, 4)),
             (BINARY_SAME, (5,)), (BINARY_SAME, (6,)), (BINARY_SAME, (7,))]
    return _finish(rng, X, terms)


def gaussian_gp(N: int, noise_var: float = 0.1, seed: int = 0):
    """GP regression with a Gaussian likelihood (test target)."""
    rng = np.random.default_rng(seed)
    X = rng.uniform(-1.0, 1.0, size=(N, 2))
    terms = [(SE_ISO, (0, 1))]
    P = 2
    eta_true = rng.standard_normal(P)
    L = np.linalg.cholesky(_gram_for_data(X, terms, eta_true, 1e-6))
    f_true = L @ rng.standard_normal(N)
    y = f_true + math.sqrt(noise_var) * rng.standard_normal(N)
    spec = ModelSpec(X=X, y=y, terms=terms, lik=LIK_GAUSSIAN, noise_var=noise_var)
    return spec, eta_true, f_true


def mean_variance(R: int, seed: int = 0, delta: float = 0.01):
    """Example 1 of Sec. 2.1: y_i = f_1(x_i) + e_i, e_i ~ N(0, delta + exp f_2(x_i)),
    with R records of two covariates x ~ N(0, I_2); f_1 ~ GP(SE-ARD) and
    f_2 ~ GP(SE-iso), each with its own hyperparameters (P = 3 + 2).  The
    latent points are stacked (f_1 at the R records, then f_2), D = 2R + 5."""
    rng = np.random.default_rng(seed)
    x = rng.standard_normal((R, 2))
    X = np.zeros((2 * R, 3))
    X[:R, :2] = x
    X[R:, :2] = x
    X[R:, 2] = 1.0
    t1, t2 = [(SE_ARD, (0, 1))], [(SE_ISO, (0, 1))]
    eta1 = rng.standard_normal(term_nparams(*t1[0]))
    eta2 = rng.standard_normal(term_nparams(*t2[0]))
    f1 = np.linalg.cholesky(_gram_for_data(x, t1, eta1, 1e-6)) @ rng.standard_normal(R)
    f2 = np.linalg.cholesky(_gram_for_data(x, t2, eta2, 1e-6)) @ rng.standard_normal(R)
    y = f1 + np.sqrt(delta + np.exp(f2)) * rng.standard_normal(R)
    spec = ModelSpec(X=X, y=np.concatenate([y, y]), terms=t1 + t2, lik=LIK_GAUSSIAN_MV,
                     delta=delta, fn_col=2, term_fns=(0, 1))
    return spec, np.concatenate([eta1, eta2]), np.concatenate([f1, f2])


BASIS_GAUSS = 0    # a one-dimensional Gaussian kernel, M sinusoidal features
BASIS_LINEAR = 1   # a linear kernel, one feature (the covariate itself)


@dataclasses.dataclass
class BasisSpec:
    """The paper's reduced-rank basis model (Sec. 2.1, Eqs. BMKL,
    Solin_representation and hpar_prior; features in the appendix on the
    reduced-rank representation), one latent function (J = 1):
        f(x_i) = sum_k sum_m a_km phi_km(x_ik) + b,
        a_km ~ N(0, c_g V_m(sigma_g)) (Gaussian-kernel covariates),
        a_k  ~ N(0, c_l)              (linear-kernel covariates, phi = x),
        b ~ N(0, bias_var), c_g, sigma_g, c_l ~ InvGamma(alpha, beta).
    q = (a in covariate order, b, c_g, sigma_g, c_l): the hyperparameters are
    sampled on their own scale (positive), as the paper writes them."""
    X: np.ndarray                     # N x dx covariates
    y: np.ndarray                     # N labels {0,1} (logit) or targets (Gaussian)
    kinds: Tuple[int, ...]            # BASIS_GAUSS / BASIS_LINEAR per covariate
    M: int = 30                       # features per Gaussian-kernel covariate
    L: float = 8.0                    # domain half-width [-L, L]
    bias_var: float = 1.0             # Sigma
    ig_alpha: Tuple[float, float, float] = (2.0, 2.0, 2.0)   # (c_g, sigma_g, c_l)
    ig_beta: Tuple[float, float, float] = (2.0, 2.0, 2.0)
    lik: int = LIK_BERNOULLI_LOGIT
    noise_var: float = 1.0
    beta: float = 1.0                 # inverse temperature on the likelihood

    def __post_init__(self):
        self.X = np.ascontiguousarray(np.asarray(self.X, dtype=np.float64))
        self.y = np.ascontiguousarray(np.asarray(self.y, dtype=np.float64))
        self.kinds = tuple(int(k) for k in self.kinds)
        if self.X.ndim != 2 or len(self.kinds) != self.X.shape[1]:
            raise ValueError("one kernel kind per covariate")
        if self.lik not in (LIK_BERNOULLI_LOGIT, LIK_GAUSSIAN):
            raise ValueError("the basis model takes the logit or Gaussian likelihood")

    @property
    def N(self) -> int:
        return self.X.shape[0]

    @property
    def dx(self) -> int:
        return self.X.shape[1]

    @property
    def n_records(self) -> int:
        return self.N

    @property
    def n_features(self) -> int:
        return sum(self.M if k == BASIS_GAUSS else 1 for k in self.kinds)

    @property
    def P(self) -> int:
        return 3

    @property
    def D(self) -> int:
        return self.n_features + 1 + 3


def basis_logistic(D_in: int, N: int = 500, seed: int = 0, M: int = 30, L: float = 8.0):
    """The simulated logistic-regression data of Sec. 2.5: x ~ N(0, 1)^D_in;
    f* = sum_k sum_m a*_km sin(pi m (x_k + L) / 2L) + b* with b* = -0.5,
    a*_km ~ N(0, c* / m) for 4 <= m <= 16 and 0 otherwise, c* set so that the
    empirical SD of f* is 1.5; labels 1 with probability sigmoid(f*).  The
    model: a Gaussian kernel with M features per covariate (d = M D_in + 4),
    alpha_theta = beta_theta = 2 for every hyperparameter, Sigma = 1."""
    rng = np.random.default_rng(seed)
    X = rng.standard_normal((N, D_in))
    m = np.arange(1, M + 1)
    z = rng.standard_normal((D_in, M)) / np.sqrt(m)
    z[:, (m < 4) | (m > 16)] = 0.0
    feats = np.sin(np.pi * m[None, None, :] * (X[:, :, None] + L) / (2.0 * L))   # N x D_in x M
    g = np.einsum("nkm,km->n", feats, z)
    c_star = (1.5 / np.std(g)) ** 2
    f = np.sqrt(c_star) * g - 0.5
    y = (rng.uniform(size=N) < 1.0 / (1.0 + np.exp(-f))).astype(np.float64)
    spec = BasisSpec(X=X, y=y, kinds=(BASIS_GAUSS,) * D_in, M=M, L=L)
    return spec, f


@dataclasses.dataclass
class ChainSettings:
    eps: float
    n_leapfrog: int       # C
    n_fixed_point: int    # K
    n_samples: int        # kept moves
    n_burnin: int         # A0
    alpha: float = 1e6
    sqrt_map: bool = False   # softabs g = sqrt(kappa^2 + lambda^2), kappa = 1/alpha

    @property
    def n_moves(self) -> int:
        return self.n_samples + self.n_burnin


# Named workloads ------------------------------------------------------------

# Step sizes: with latent f as coordinates and jitter 1e-6 the posterior is
# stiff in the kernel hyperparameters (K^-1 reaches 1/jitter and moves
# exponentially with the lengthscales), and K plain fixed-point iterations of
# the implicit leapfrog diverge at eps = 0.1 (d = 34) or 0.05 (multiple-kernel):
# the FP64 reference's energy error overflows in the first move.  For the
# D = 1038 model the FP64 reference also leaves the domain within the first
# move at eps = 0.003 (energy error -31.7 after 8 leapfrogs from q = 0, non-
# finite after 9), while eps = 0.001 -- the step size of the paper's own runs
# (Sec. 2.5) -- integrates 20 leapfrogs with converged fixed-point iterations.
# The cost of a leapfrog does not depend on eps beyond the number of Jacobi
# sweeps of the warm-started eigendecompositions.
EPS_STATED = {"gp_logistic_d34": 0.1, "gp_logistic_ard_d261": 0.05, "propensity_mkl_d1038": 0.05}


def start_point(spec):
    """The chains' start: q = 0 for the latent models; a = 0, b = 0 and every
    hyperparameter 1 for the basis model (as the paper starts, Sec. 2.5)."""
    q = np.zeros(spec.D)
    if isinstance(spec, BasisSpec):
        q[-3:] = 1.0
    return q


def workload(name: str, seed: int = 0):
    """Return (spec, settings) for a named workload."""
    if name == "gp_logistic_d34":
        spec, _, _ = gp_logistic_2d(32, seed)
        return spec, ChainSettings(eps=0.01, n_leapfrog=10, n_fixed_point=6,
                                   n_samples=200, n_burnin=67)
    if name == "gp_logistic_ard_d261":
        spec, _, _ = gp_logistic_ard4(256, seed)
        return spec, ChainSettings(eps=0.003, n_leapfrog=20, n_fixed_point=6,
                                   n_samples=1000, n_burnin=334)
    if name == "propensity_mkl_d1038":
        spec, _, _ = propensity_mkl(1024, seed)
        return spec, ChainSettings(eps=0.001, n_leapfrog=20, n_fixed_point=6,
                                   n_samples=200, n_burnin=67)
    if name in ("basis_logistic_d34", "basis_logistic_d484"):
        # the paper's own model and data recipe (Sec. 2.5): C = 100, eps = 1e-3
        spec, _ = basis_logistic(1 if name.endswith("d34") else 16, seed=seed)
        return spec, ChainSettings(eps=0.001, n_leapfrog=100, n_fixed_point=6,
                                   n_samples=9600 - 2400, n_burnin=2400, alpha=1.0,
                                   sqrt_map=True)
    if name == "mean_variance_d1029":
        # Example 1 of Sec. 2.1 at R = 512 records: 1024 latent values + 5
        spec, _, _ = mean_variance(512, seed)
        return spec, ChainSettings(eps=0.001, n_leapfrog=20, n_fixed_point=6,
                                   n_samples=200, n_burnin=67)
    raise KeyError(name)


def tempered_ladder(n_chains: int = 64, seed: int = 0):
    """Tempered chains for evidence estimation: beta_k = (k/(n-1))^5 and a
    chain dimension drawn uniformly from {66,130,258,514} (one dataset per D)."""
    rng = np.random.default_rng(seed)
    dims = rng.choice(np.array([66, 130, 258, 514]), size=n_chains)
    betas = (np.arange(n_chains) / (n_chains - 1)) ** 5
    data = {}
    for D in sorted(set(int(d) for d in dims)):
        data[D], _, _ = gp_logistic_2d(D - 2, seed)
    specs = []
    for k in range(n_chains):
        base = data[int(dims[k])]
        specs.append(dataclasses.replace(base, beta=float(betas[k])))
    return specs, dims, betas
