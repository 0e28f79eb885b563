"""Reference oracle (test infrastructure only).

Plain FP64 CPU implementation of what the GPU path computes.  Only the test
suite, the smoke check and the benchmark's CPU-baseline leg may import it;
the GPU library and its Python binding never do.  It shares no code with the
GPU library: the compiled part (``oracle.c``) defines the field, the
finite-volume system, the banded Cholesky solve, the quantity of interest,
the Algorithm 2.1 refinement reference and the adjoint gradient; this module
adds the ctypes marshalling and the statistical layer (sec. 4.1 estimator,
the accuracy rule of sec. 4.5 and Algorithm 4.1 of sec. 4.3).

Functions and the passage each follows:
  kl_roots / kl_basis      -- KL expansion of the separable exponential
                              covariance (field of the workloads)
  trig_basis               -- the paper's own trigonometric field (sec. 5.1)
  solve_batch              -- exact discrete solution, Q = integral of u
                              (sec. 5.1 QoI)
  ir_f32_batch             -- Algorithm 2.1 with (u_f,u_s,u,u_r) = (s,s,d,d)
  ir_lowp_batch            -- the same with the factor and substitutions of
                              the scaled system simulated in FP16, BF16 or
                              FP32 (every operation rounded, Sec. 2.1's
                              simulated low precision)
  grad_batch               -- adjoint dQ/dxi (not in the paper; exact
                              derivative of the discrete Q)
  accuracy_targets         -- delta_l of sec. 4.5 (sqrt(k_p) h_l^2, k_p h_L^2)
  accuracy_targets_rates   -- the general precision choice of sec. 4.3
  level_estimates          -- Y-hat_l and s_l^2 of sec. 4.1
  adaptive_mpml            -- Algorithm 4.1 (sec. 4.3)
  cost_ratio_bound         -- bound of the cost-savings corollary, sec. 4.4
  mlmcmc                   -- multilevel MCMC (the extension named in the
                              remark on other sampling methods, sec. 4):
                              pCN chains on level 0, two-level chains with
                              an independence proposal from a coarse chain
  mimc                     -- multi-index Monte Carlo (the second sampler of
                              that remark): sample means of the mixed
                              differences over a set of (grid, truncation)
                              indices
"""
import ctypes
import math
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_LIB_PATH = os.path.join(_HERE, "liboracle.so")
_lib = None


def build(force=True):
    """Compile oracle.c into liboracle.so with gcc (OpenMP over samples)."""
    src = os.path.join(_HERE, "oracle.c")
    cmd = ["gcc", "-O2", "-fopenmp", "-shared", "-fPIC", "-o", _LIB_PATH + ".tmp", src, "-lm"]
    if force or not os.path.exists(_LIB_PATH):
        subprocess.check_call(cmd)
        os.replace(_LIB_PATH + ".tmp", _LIB_PATH)
    return _LIB_PATH


def _load():
    global _lib
    if _lib is None:
        src = os.path.join(_HERE, "oracle.c")
        if not os.path.exists(_LIB_PATH) or os.path.getmtime(src) > os.path.getmtime(_LIB_PATH):
            build(force=True)
        lib = ctypes.CDLL(_LIB_PATH)
        D = ctypes.POINTER(ctypes.c_double)
        I = ctypes.POINTER(ctypes.c_int)
        c_int, c_double = ctypes.c_int, ctypes.c_double
        lib.oracle_kl_roots.argtypes = [c_double, c_int, D]
        lib.oracle_kl_modes.argtypes = [c_double, c_int, c_int, I, I]
        lib.oracle_kl_basis.argtypes = [c_int, c_int, c_double, c_double, D]
        lib.oracle_kl_mu.argtypes = [c_double, c_double]
        lib.oracle_kl_mu.restype = c_double
        lib.oracle_kl_phi1d.argtypes = [c_double, c_double, c_double]
        lib.oracle_kl_phi1d.restype = c_double
        lib.oracle_solve_batch.argtypes = [c_int, c_int, D, c_int, D, D, c_double, D, D, D]
        lib.oracle_relres_batch.argtypes = [c_int, c_int, D, c_int, D, c_double, D, D]
        lib.oracle_ir_f32_batch.argtypes = [c_int, c_int, D, c_int, D, c_double, c_double, c_int,
                                            D, I, D]
        lib.oracle_ir_lowp_batch.argtypes = [c_int, c_int, D, c_int, D, c_double, c_double, c_int, c_int,
                                             D, I, D]
        lib.oracle_round_lowp.argtypes = [c_double, c_int]
        lib.oracle_round_lowp.restype = c_double
        lib.oracle_grad_batch.argtypes = [c_int, c_int, D, c_int, D, c_double, D, D, D]
        lib.oracle_energy.argtypes = [c_int, c_int, D, D, D]
        lib.oracle_energy.restype = c_double
        lib.oracle_dense_matrix.argtypes = [c_int, c_int, D, D, D]
        lib.oracle_band_matrix.argtypes = [c_int, c_int, D, D, D]
        lib.oracle_set_threads.argtypes = [c_int]
        lib.oracle_set_threads.restype = None
        lib.oracle_set_disc.argtypes = [c_int]
        lib.oracle_set_disc.restype = None
        lib.oracle_num_threads.restype = c_int
        _lib = lib
    return _lib


def _p(a):
    if a is None:
        return None
    return a.ctypes.data_as(ctypes.POINTER(ctypes.c_double))


def _pi(a):
    return a.ctypes.data_as(ctypes.POINTER(ctypes.c_int))


def _f64(a):
    return np.ascontiguousarray(a, dtype=np.float64)


def num_threads():
    return _load().oracle_num_threads()


# ---------------------------------------------------------------- KL field

def kl_roots(corr_len, M=64):
    w = np.zeros(M)
    if _load().oracle_kl_roots(corr_len, M, _p(w)):
        raise RuntimeError("bracketing failed")
    return w


def kl_mu(corr_len, w):
    return np.array([_load().oracle_kl_mu(corr_len, float(x)) for x in np.atleast_1d(w)])


def kl_phi1d(corr_len, w, x):
    return np.array([_load().oracle_kl_phi1d(corr_len, float(w), float(t)) for t in np.atleast_1d(x)])


def kl_modes(corr_len, K, M=64):
    mi = np.zeros(K, dtype=np.int32)
    mj = np.zeros(K, dtype=np.int32)
    rc = _load().oracle_kl_modes(corr_len, K, M, _pi(mi), _pi(mj))
    if rc:
        raise RuntimeError("mode selection failed (%d)" % rc)
    return mi, mj


def kl_basis(n, K, sigma2, corr_len):
    """Phi[(n+1)^2, K] on the nodes of the n x n grid (node p = iy*(n+1)+ix)."""
    Phi = np.zeros(((n + 1) * (n + 1), K))
    if _load().oracle_kl_basis(n, K, sigma2, corr_len, _p(Phi)):
        raise RuntimeError("KL basis failed")
    return Phi


def trig_basis(n, K, sigma2, q):
    """Phi[(n+1)^2, K] of the trigonometric field of sec. 5.1 (the random
    coefficient's exponent sum_{j<=s} omega_j j^-q sin(2 pi j x1) cos(2 pi j x2),
    omega_j ~ N(0, sigma^2)), written for xi_j = omega_j / sigma ~ N(0, 1):
    column j-1 is sigma j^-q sin(2 pi j x) cos(2 pi j y) on the nodes
    (node p = iy*(n+1)+ix), j = 1..K (= s)."""
    t = np.arange(n + 1) / n
    x = np.tile(t, n + 1)          # ix fastest
    y = np.repeat(t, n + 1)
    Phi = np.empty(((n + 1) * (n + 1), K))
    for j in range(1, K + 1):
        Phi[:, j - 1] = math.sqrt(sigma2) * j ** (-float(q)) * np.sin(2 * math.pi * j * x) * np.cos(2 * math.pi * j * y)
    return Phi


# ---------------------------------------------------------------- solves

def solve_batch(n, Phi, xi, f=1.0, a_nodes=None, rhs_nodal=None, want_u=False):
    """Exact FP64 solve; returns Q[S] (and u[S, (n-1)^2] if want_u)."""
    K = Phi.shape[1] if Phi is not None else 0
    if a_nodes is not None:
        a_nodes = _f64(np.atleast_2d(a_nodes))
        S = a_nodes.shape[0]
    else:
        xi = _f64(np.atleast_2d(xi))
        S = xi.shape[0]
    Q = np.zeros(S)
    u = np.zeros((S, (n - 1) ** 2)) if want_u else None
    rc = _load().oracle_solve_batch(n, K, _p(_f64(Phi)) if Phi is not None else None, S,
                                    _p(xi) if a_nodes is None else None, _p(a_nodes), f,
                                    _p(_f64(rhs_nodal)) if rhs_nodal is not None else None,
                                    _p(Q), _p(u))
    if rc:
        raise RuntimeError("Cholesky breakdown in sample %d" % (rc - 1))
    return (Q, u) if want_u else Q


def relres_batch(n, Phi, xi, x, f=1.0):
    xi = _f64(np.atleast_2d(xi))
    x = _f64(np.atleast_2d(x))
    rr = np.zeros(xi.shape[0])
    _load().oracle_relres_batch(n, Phi.shape[1], _p(_f64(Phi)), xi.shape[0], _p(xi), f, _p(x), _p(rr))
    return rr


def ir_f32_batch(n, Phi, xi, delta, imax=10, f=1.0):
    """Algorithm 2.1 with a single-precision factor; returns (Q, trips, relres, n_fail)."""
    xi = _f64(np.atleast_2d(xi))
    S = xi.shape[0]
    Q = np.zeros(S)
    trips = np.zeros(S, dtype=np.int32)
    rr = np.zeros(S)
    nf = _load().oracle_ir_f32_batch(n, Phi.shape[1], _p(_f64(Phi)), S, _p(xi), f, delta, imax,
                                     _p(Q), _pi(trips), _p(rr))
    return Q, trips, rr, nf


LOWP_FORMATS = {"f16": 0, "bf16": 1, "f32": 2}


def round_lowp(v, fmt):
    """v rounded to "f16", "bf16" or "f32" (nearest, ties to even) as the
    simulated low precision rounds every result."""
    return _load().oracle_round_lowp(float(v), LOWP_FORMATS[fmt])


def ir_lowp_batch(n, Phi, xi, delta, fmt, imax=10, f=1.0):
    """Algorithm 2.1 with the factorisation and substitutions of the scaled
    system simulated in a low precision (every operation rounded: "f16",
    "bf16" or "f32"), residual and update in FP64; returns (Q, trips, relres,
    n_fail), trips -1 for a factorisation that broke down."""
    xi = _f64(np.atleast_2d(xi))
    S = xi.shape[0]
    Q = np.zeros(S)
    trips = np.zeros(S, dtype=np.int32)
    rr = np.zeros(S)
    nf = _load().oracle_ir_lowp_batch(n, Phi.shape[1], _p(_f64(Phi)), S, _p(xi), f, delta, imax,
                                      LOWP_FORMATS[fmt], _p(Q), _pi(trips), _p(rr))
    return Q, trips, rr, nf


def grad_batch(n, Phi, xi, f=1.0, want_gz=False, want_lambda=False):
    xi = _f64(np.atleast_2d(xi))
    S, K = xi.shape
    g = np.zeros((S, K))
    gz = np.zeros((S, (n + 1) ** 2)) if want_gz else None
    lam = np.zeros((S, (n - 1) ** 2)) if want_lambda else None
    rc = _load().oracle_grad_batch(n, K, _p(_f64(Phi)), S, _p(xi), f, _p(g), _p(gz), _p(lam))
    if rc:
        raise RuntimeError("Cholesky breakdown in sample %d" % (rc - 1))
    out = [g]
    if want_gz:
        out.append(gz)
    if want_lambda:
        out.append(lam)
    return out[0] if len(out) == 1 else tuple(out)


def energy(n, Phi, xi, u):
    return _load().oracle_energy(n, Phi.shape[1], _p(_f64(Phi)), _p(_f64(xi)), _p(_f64(u)))


def band_matrix(n, Phi, xi):
    """A of one sample in LAPACK lower band form ab[d, j] = A[j+d, j], d = 0..n-1."""
    m = n - 1
    N, bw = m * m, m
    Ab = np.zeros((N, bw + 1))
    _load().oracle_band_matrix(n, Phi.shape[1], _p(_f64(Phi)), _p(_f64(np.atleast_2d(xi)[0])), _p(Ab))
    ab = np.zeros((bw + 1, N))
    for d in range(bw + 1):
        ab[d, :N - d] = Ab[d:, d]
    return ab


def set_disc(d):
    """Edge rule of every later assembly: 0 finite volumes (harmonic mean of
    the edge's end nodes), 1 P1 elements on right triangles (sec. 3)."""
    if d not in (0, 1):
        raise ValueError("disc is 0 or 1")
    _load().oracle_set_disc(int(d))


class disc_rule:
    """Context manager: assemble with edge rule d inside the block."""

    def __init__(self, d):
        self.d = d

    def __enter__(self):
        set_disc(self.d)
        return self

    def __exit__(self, *exc):
        set_disc(0)
        return False


def set_threads(k):
    """Threads of the oracle's later OpenMP regions."""
    _load().oracle_set_threads(int(k))


def dense_matrix(n, Phi, xi):
    N = (n - 1) ** 2
    A = np.zeros((N, N))
    _load().oracle_dense_matrix(n, Phi.shape[1], _p(_f64(Phi)), _p(_f64(xi)), _p(A))
    return A


# ---------------------------------------------------------------- MLMC layer

def accuracy_targets(h, L, k_p=0.05):
    """delta_l, l = 0..L, from the rule of sec. 4.5:
    delta_l = sqrt(k_p) h_l^2 for l < L and delta_L = k_p h_L^2."""
    return [math.sqrt(k_p) * h[l] ** 2 if l < L else k_p * h[l] ** 2 for l in range(L + 1)]


def accuracy_targets_rates(h, L, k_p, alpha1, beta1, alpha2=1.0, beta2=2.0):
    """delta_l, l = 0..L, from the general precision-choice equation of
    sec. 4.3 with bias O(h^alpha1 + delta^alpha2) and variance
    O(h^beta1 + delta^beta2):
    delta_l = (k_p h_l^beta1)^(1/beta2) for l < L and
    delta_L = min((k_p h_L^beta1)^(1/beta2), (k_p h_L^alpha1)^(1/alpha2)).
    The exponents of delta default to those of the error lemma of sec. 4.5
    (1 in the bias, 2 in the variance)."""
    out = []
    for l in range(L + 1):
        ev = (k_p * h[l] ** beta1) ** (1.0 / beta2)
        out.append(ev if l < L else min(ev, (k_p * h[l] ** alpha1) ** (1.0 / alpha2)))
    return out


def level_estimates(y):
    """Y-hat_l = mean and s_l^2 = (1/N_l) sum (Y - Y-hat)^2 (sec. 4.1)."""
    y = np.asarray(y, dtype=np.float64)
    yhat = y.sum() / y.size
    return yhat, ((y - yhat) ** 2).sum() / y.size


def factor_cost(n, gamma=4.0):
    """Deterministic cost units of one grid solve: (n-1)^gamma (gamma = 4:
    the flops of the factor)."""
    return float(n - 1) ** gamma


def level_cost(n0, l, m=2, gamma=4.0):
    c = factor_cost(n0 * m ** l, gamma)
    if l > 0:
        c += factor_cost(n0 * m ** (l - 1), gamma)
    return c


def cost_ratio_bound(q, beta, gamma, m=2):
    """Asymptotic bound q + m^((gamma-beta)/2) (1 - q) of the cost-savings corollary (sec. 4.4)."""
    r = m ** ((gamma - beta) / 2.0)
    return q + r * (1.0 - q)


def adaptive_mpml(sample_fn, n0, tol, L_max, n_init=1000, m=2, alpha=2.0, k_p=0.05, mixed=True,
                  max_rounds=100):
    """Algorithm 4.1 (adaptive MPML), sec. 4.3, in the paper's order.

    sample_fn(level, first, count, delta_fine, delta_coarse) -> array Y of the
    new samples (Y_0 = Q_0; Y_l = Q_l - Q_{l-1} on one shared xi row).  With
    mixed=False the accuracy step is skipped (standard MLMC) and deltas are 0.
    Readings: r = 1 in the bias test; V_l = s_l^2; C_l from level_cost; the
    coarse partner of Y_l is solved to delta_{l-1}; returns once the bias test
    and the variance test both hold and no level needs more samples.
    """
    h = [1.0 / (n0 * m ** l) for l in range(L_max + 1)]
    L = 1
    N = [n_init, n_init]
    done = [0, 0]
    s1 = [0.0, 0.0]
    s2 = [0.0, 0.0]
    bias_c = (m ** alpha - 1.0) / math.sqrt(2.0) * tol
    rounds = 0
    history = []
    while L <= L_max and rounds < max_rounds:
        rounds += 1
        eps = accuracy_targets(h, L, k_p) if mixed else [0.0] * (L + 1)
        for l in range(L + 1):
            dn = max(0, int(N[l]) - done[l])
            if dn > 0:
                y = np.asarray(sample_fn(l, done[l], dn, eps[l], eps[l - 1] if l > 0 else 0.0))
                s1[l] += float(y.sum())
                s2[l] += float((y * y).sum())
                done[l] += dn
        yhat = [s1[l] / done[l] for l in range(L + 1)]
        var = [max(s2[l] / done[l] - yhat[l] ** 2, 0.0) for l in range(L + 1)]
        C = [level_cost(n0, l, m) for l in range(L + 1)]
        tot = sum(math.sqrt(var[k] * C[k]) for k in range(L + 1))
        N = [max(done[l], int(math.ceil(math.sqrt(var[l] / C[l]) * 2.0 / tol ** 2 * tot)))
             for l in range(L + 1)]
        history.append(dict(L=L, N=list(N), done=list(done), yhat=list(yhat), var=list(var)))
        if abs(yhat[L]) > bias_c and L < L_max:
            L += 1
            N.append(n_init)
            done.append(0)
            s1.append(0.0)
            s2.append(0.0)
            continue
        need_more = any(N[l] > done[l] for l in range(L + 1))
        var_ok = sum(var[l] / done[l] for l in range(L + 1)) <= tol ** 2 / 2.0
        if not need_more:
            return dict(estimate=sum(yhat), L=L, N=list(done), yhat=yhat, s2=var,
                        bias_ok=abs(yhat[L]) <= bias_c, var_ok=var_ok, rounds=rounds,
                        history=history)
    raise RuntimeError("adaptive MPML did not terminate")


# ---------------------------------------------------------------- multilevel MCMC

def pde_forward(n, Phi, obs, noise_sd, disc=0):
    """forward(xi[C, K]) -> (Q, log-likelihood) of the discrete PDE on grid n:
    log L = -sum_j (d_j - u(x_j))^2 / (2 noise_sd^2) at the observation nodes
    obs = [(x, y, d)] (nodes of the grid)."""
    m = n - 1

    def f(xi):
        with disc_rule(disc):
            q, u = solve_batch(n, Phi, xi, want_u=True)
        ll = np.zeros(xi.shape[0])
        for x, y, d in obs:
            ix, iy = int(round(x * n)), int(round(y * n))
            ll -= (d - u[:, (iy - 1) * m + (ix - 1)]) ** 2 / (2.0 * noise_sd ** 2)
        return q, ll
    return f


def mlmcmc(forward, L, chains, K, steps, burn_in, subsample, beta, normals):
    """Multilevel MCMC for E_{pi_L}[Q] = E_{pi_0}[Q_0] + sum_l E[Q_l - Q_{l-1}],
    written from Dodwell, Ketelsen, Scheichl and Teckentrup's method (the
    sampler the remark on other sampling methods names), every chain started
    at xi = 0, the first burn_in steps not recorded:
      level 0: preconditioned Crank-Nicolson, xi' = sqrt(1 - beta^2) xi + beta w,
        accepted when Phi(z) < L_0(xi') / L_0(xi) (a prior-reversible proposal);
      level l >= 1: a pCN chain on pi_{l-1} advanced `subsample` steps, whose
        state is proposed to a chain on pi_l and accepted when
        Phi(z) < L_l(xi') L_{l-1}(xi) / (L_l(xi) L_{l-1}(xi')) (an independence
        proposal drawn from pi_{l-1}); Y_l = Q_l(fine state) - Q_{l-1}(coarse state).
    forward(l, xi) -> (Q, log L) on level l; normals(stream, first, count, k)
    -> [count, k] standard normals of the counter-based generator, streams
    4096 + 8 l + {0 fine proposals, 1 coarse proposals, 2 fine, 3 coarse
    acceptance}, index step * chains + chain (coarse: (step * subsample + s)
    * chains + chain).  Returns per-level means, chain-mean variances of the
    means, acceptance rates and the estimate."""
    C = chains
    c1 = math.sqrt(1.0 - beta * beta)

    def accept(log_a, z, ll_new):
        u = 0.5 * np.array([math.erfc(-v / math.sqrt(2.0)) for v in z])
        with np.errstate(over="ignore"):
            return np.isfinite(ll_new) & ((log_a >= 0.0) | (u < np.exp(np.minimum(log_a, 0.0))))

    out = dict(Yhat=[], var_mean=[], accept=[], accept_coarse=[])
    for l in range(L + 1):
        base = 4096 + 8 * l
        T = burn_in + steps[l]
        th = np.zeros((C, K))
        qf, llf = forward(l, th)
        if l > 0:
            tc = np.zeros((C, K))
            qc, llc = forward(l - 1, tc)
            llcf = llc.copy()
        sums = np.zeros(C)
        acc = np.zeros(C)
        acc_c = np.zeros(C)
        for k in range(T):
            rec = k >= burn_in
            if l == 0:
                prop = c1 * th + beta * normals(base + 0, k * C, C, K)
                qp, llp = forward(0, prop)
                a = accept(llp - llf, normals(base + 2, k * C, C, 1)[:, 0], llp)
                th[a], llf[a], qf[a] = prop[a], llp[a], qp[a]
                if rec:
                    acc += a
                    sums += qf
                continue
            for sub in range(subsample):
                idx = (k * subsample + sub) * C
                prop = c1 * tc + beta * normals(base + 1, idx, C, K)
                qp, llp = forward(l - 1, prop)
                a = accept(llp - llc, normals(base + 3, idx, C, 1)[:, 0], llp)
                tc[a], llc[a], qc[a] = prop[a], llp[a], qp[a]
                if rec:
                    acc_c += a
            prop = tc.copy()
            qp, llp = forward(l, prop)
            a = accept((llp - llf) - (llc - llcf), normals(base + 2, k * C, C, 1)[:, 0], llp)
            th[a], llf[a], qf[a], llcf[a] = prop[a], llp[a], qp[a], llc[a]
            if rec:
                acc += a
                sums += qf - qc
        means = sums / steps[l]
        out["Yhat"].append(float(means.mean()))
        out["var_mean"].append(float(means.var(ddof=1) / C) if C > 1 else 0.0)
        out["accept"].append(float(acc.sum() / (C * steps[l])))
        out["accept_coarse"].append(float(acc_c.sum() / (C * steps[l] * subsample)) if l else 0.0)
    out["estimate"] = float(sum(out["Yhat"]))
    return out


def mimc(indices, N, K0, K, solve, normals):
    """Multi-index Monte Carlo, written from the definition of Haji-Ali, Nobile
    and Tempone's estimator (the second sampler of the remark on other
    sampling methods at the end of sec. 4): E[Q] ~ sum over the index set of
    the sample mean of the mixed difference
      D_(l,k)(xi) = Q_(l,k) - Q_(l-1,k) - Q_(l,k-1) + Q_(l-1,k-1),
    terms with a negative index left out, over N[i] independent samples of
    index i = (l, k); Q_(l,k)(xi) is the level-l quantity of xi with the
    coefficients from mode min(K, K0 2^k) on set to zero (the field's modes
    ordered by decreasing variance).  solve(l, xi) -> Q_l for the rows of xi;
    normals(i, count) -> [count, K] samples of index i.  Returns the
    per-index means and variances (N - 1 normalisation) and their sums."""
    out = dict(mean=[], var=[])
    for i, (l, k) in enumerate(indices):
        xi = np.asarray(normals(i, N[i]), dtype=np.float64)
        d = np.zeros(N[i])
        for t in (0, 1):              # truncation k - t
            if k - t < 0:
                continue
            xm = xi.copy()
            xm[:, min(K, K0 << (k - t)):] = 0.0
            for g in (0, 1):          # grid l - g
                if l - g < 0:
                    continue
                d += (-1.0) ** (t + g) * np.asarray(solve(l - g, xm), dtype=np.float64)
        out["mean"].append(float(d.mean()))
        out["var"].append(float(d.var(ddof=1)))
    out["estimate"] = float(sum(out["mean"]))
    out["var_estimate"] = float(sum(v / n for v, n in zip(out["var"], N)))
    return out

