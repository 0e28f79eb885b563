"""Python binding of libmlmc (argument marshalling only).

Every step of the sample solve runs in the HIP library; this module only
allocates device buffers with PyTorch, passes their pointers and the current
HIP stream through the C ABI declared in include/mlmc.h, and converts
results.  There is no CPU fallback: if the library is missing, or no GPU is
visible, the calls raise.
"""
import ctypes
import dataclasses
import os

import torch  # loads PyTorch's HIP runtime first; libmlmc binds to the same one

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libmlmc.so")

MLMC_OK, MLMC_ENOCONV = 0, 1
MLMC_EINVAL, MLMC_ENOMEM, MLMC_EHIP, MLMC_ENOTIMPL = -1, -2, -3, -4
DTYPES = {"f64": 0, "f32": 1, "bf16": 2, "f16": 3, "fp8": 4}
SOLVERS = {"direct": 0, "direct_ir": 1, "minres": 2, "minres_ir": 3, "mgcg": 4}
ST_CONVERGED, ST_PROMOTED, ST_NONFINITE, ST_IMAX = 1, 2, 4, 8

EXPORTS = ["mlmc_create", "mlmc_destroy", "mlmc_last_error", "mlmc_level_cells",
           "mlmc_accuracy_targets", "mlmc_get_kl_basis", "mlmc_workspace_bytes", "mlmc_fill_xi",
           "mlmc_solve", "mlmc_sample_level", "mlmc_estimate", "mlmc_grad", "mlmc_profile",
           "mlmc_profile_read", "mlmc_levels_workspace_bytes", "mlmc_sample_levels", "mlmc_autotune",
           "mlmc_sample_level_noalloc", "mlmc_set_seed", "mlmc_mcmc", "mlmc_mimc", "mlmc_estimate_resumable"]
NOALLOC_SCRATCH_BYTES = 64 << 20


class MLMCError(RuntimeError):
    pass


class _Config(ctypes.Structure):
    _fields_ = [("n0", ctypes.c_int32), ("m", ctypes.c_int32), ("L_max", ctypes.c_int32),
                ("K", ctypes.c_int32), ("sigma2", ctypes.c_double), ("corr_len", ctypes.c_double),
                ("f", ctypes.c_double), ("k_p", ctypes.c_double), ("alpha", ctypes.c_double),
                ("beta", ctypes.c_double), ("gamma", ctypes.c_double),
                ("ir_max_iter", ctypes.c_int32), ("minres_max_iter", ctypes.c_int32),
                ("seed", ctypes.c_uint64), ("field", ctypes.c_int32), ("field_q", ctypes.c_double),
                ("disc", ctypes.c_int32), ("std_eps", ctypes.c_double)]


class _LevelOpts(ctypes.Structure):
    _fields_ = [("factor_dtype", ctypes.c_int), ("solver", ctypes.c_int),
                ("eps_fine", ctypes.c_double), ("eps_coarse", ctypes.c_double),
                ("promote", ctypes.c_int32)]


class _LevelStats(ctypes.Structure):
    _fields_ = [("n", ctypes.c_int64), ("sum_y", ctypes.c_double), ("sum_y2", ctypes.c_double),
                ("sum_qf", ctypes.c_double), ("sum_qc", ctypes.c_double),
                ("n_promoted", ctypes.c_int64), ("n_noconv", ctypes.c_int64),
                ("mean_iters", ctypes.c_double), ("gpu_ms", ctypes.c_double),
                ("mean_iters_coarse", ctypes.c_double)]


class _Result(ctypes.Structure):
    _fields_ = [("estimate", ctypes.c_double), ("var_est", ctypes.c_double),
                ("L", ctypes.c_int32), ("converged", ctypes.c_int32),
                ("N", ctypes.c_int64 * 16), ("Yhat", ctypes.c_double * 16),
                ("s2", ctypes.c_double * 16), ("C", ctypes.c_double * 16),
                ("eps", ctypes.c_double * 16), ("wall_s", ctypes.c_double),
                ("gpu_ms", ctypes.c_double), ("n_promoted", ctypes.c_int64 * 16),
                ("n_noconv", ctypes.c_int64 * 16)]


class _EstimateState(ctypes.Structure):
    _fields_ = [("L", ctypes.c_int32), ("rounds", ctypes.c_int32), ("N", ctypes.c_int64 * 16),
                ("done", ctypes.c_int64 * 16), ("s1", ctypes.c_double * 16), ("s2", ctypes.c_double * 16),
                ("n_promoted", ctypes.c_int64 * 16), ("n_noconv", ctypes.c_int64 * 16),
                ("gpu_ms", ctypes.c_double), ("tol", ctypes.c_double), ("n_init", ctypes.c_int32),
                ("mixed", ctypes.c_int32), ("solver", ctypes.c_int32), ("dtype", ctypes.c_int32 * 16),
                ("seed", ctypes.c_uint64)]


def _state_to_dict(st):
    """A plain (JSON-serialisable) copy of an estimator state."""
    d = {}
    for name, typ in _EstimateState._fields_:
        v = getattr(st, name)
        d[name] = list(v) if hasattr(typ, "_length_") else v
    return d


def _state_from_dict(d):
    st = _EstimateState()
    for name, typ in _EstimateState._fields_:
        if hasattr(typ, "_length_"):
            getattr(st, name)[:] = list(d[name])
        else:
            setattr(st, name, d[name])
    return st


class _MCMCConfig(ctypes.Structure):
    _fields_ = [("L", ctypes.c_int32), ("chains", ctypes.c_int32), ("steps", ctypes.c_int32 * 16),
                ("burn_in", ctypes.c_int32), ("subsample", ctypes.c_int32), ("pcn_beta", ctypes.c_double),
                ("noise_sd", ctypes.c_double), ("n_obs", ctypes.c_int32),
                ("obs_x", ctypes.c_double * 64), ("obs_y", ctypes.c_double * 64),
                ("obs_value", ctypes.c_double * 64), ("opts", _LevelOpts * 16), ("seed", ctypes.c_uint64)]


class _MCMCResult(ctypes.Structure):
    _fields_ = [("estimate", ctypes.c_double), ("Yhat", ctypes.c_double * 16),
                ("var_mean", ctypes.c_double * 16), ("accept", ctypes.c_double * 16),
                ("accept_coarse", ctypes.c_double * 16), ("solves", ctypes.c_int64),
                ("wall_s", ctypes.c_double)]


class _MIMCConfig(ctypes.Structure):
    _fields_ = [("n_idx", ctypes.c_int32), ("idx_l", ctypes.c_int32 * 64), ("idx_k", ctypes.c_int32 * 64),
                ("N", ctypes.c_int64 * 64), ("K0", ctypes.c_int32), ("opts", _LevelOpts * 64),
                ("seed", ctypes.c_uint64)]


class _MIMCResult(ctypes.Structure):
    _fields_ = [("estimate", ctypes.c_double), ("var_estimate", ctypes.c_double),
                ("mean", ctypes.c_double * 64), ("var", ctypes.c_double * 64),
                ("n_promoted", ctypes.c_int64 * 64), ("n_noconv", ctypes.c_int64 * 64),
                ("solves", ctypes.c_int64), ("wall_s", ctypes.c_double)]


_lib = None


def load_library():
    """Load libmlmc.so (raises if it has not been built)."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH):
        raise MLMCError("libmlmc.so is not built (run __graft_entry__.build())")
    lib = ctypes.CDLL(LIB_PATH)
    vp, i32, i64, dbl = ctypes.c_void_p, ctypes.c_int32, ctypes.c_int64, ctypes.c_double
    lib.mlmc_create.argtypes = [ctypes.POINTER(_Config), ctypes.POINTER(vp)]
    lib.mlmc_destroy.argtypes = [vp]
    lib.mlmc_last_error.argtypes = [vp]
    lib.mlmc_last_error.restype = ctypes.c_char_p
    lib.mlmc_level_cells.argtypes = [vp, i32]
    lib.mlmc_level_cells.restype = i32
    lib.mlmc_accuracy_targets.argtypes = [vp, i32, ctypes.POINTER(dbl)]
    lib.mlmc_get_kl_basis.argtypes = [vp, i32, vp, vp]
    lib.mlmc_workspace_bytes.argtypes = [vp, i32, i64, ctypes.POINTER(_LevelOpts)]
    lib.mlmc_workspace_bytes.restype = ctypes.c_size_t
    lib.mlmc_fill_xi.argtypes = [vp, i32, i64, i64, vp, vp]
    lib.mlmc_set_seed.argtypes = [vp, ctypes.c_uint64]
    lib.mlmc_solve.argtypes = [vp, i32, i64, vp, ctypes.POINTER(_LevelOpts), vp, ctypes.c_size_t,
                               vp, vp, vp, vp, vp]
    lib.mlmc_sample_level.argtypes = [vp, i32, i64, vp, ctypes.POINTER(_LevelOpts), vp,
                                      ctypes.c_size_t, vp, vp, vp, vp, ctypes.POINTER(_LevelStats), vp]
    lib.mlmc_sample_level_noalloc.argtypes = [vp, i32, i64, vp, ctypes.POINTER(_LevelOpts), vp, vp,
                                              vp, vp, ctypes.POINTER(_LevelStats), vp]
    lib.mlmc_estimate.argtypes = [vp, dbl, i32, ctypes.POINTER(ctypes.c_int), ctypes.c_int, i32,
                                  ctypes.POINTER(_Result), vp]
    lib.mlmc_grad.argtypes = [vp, i32, i64, vp, vp, ctypes.POINTER(_LevelOpts), dbl, vp,
                              ctypes.c_size_t, vp, vp]
    lib.mlmc_levels_workspace_bytes.argtypes = [vp, i32, ctypes.POINTER(i32), ctypes.POINTER(i64),
                                                ctypes.POINTER(_LevelOpts)]
    lib.mlmc_levels_workspace_bytes.restype = ctypes.c_size_t
    lib.mlmc_sample_levels.argtypes = [vp, i32, ctypes.POINTER(i32), ctypes.POINTER(i64),
                                       ctypes.POINTER(vp), ctypes.POINTER(_LevelOpts), vp,
                                       ctypes.c_size_t, ctypes.POINTER(vp), ctypes.POINTER(_LevelStats),
                                       i32, vp]
    lib.mlmc_autotune.argtypes = [vp, i32, i64, vp, ctypes.POINTER(_LevelOpts), vp, ctypes.c_size_t,
                                  ctypes.POINTER(i32), vp]
    lib.mlmc_mcmc.argtypes = [vp, ctypes.POINTER(_MCMCConfig), ctypes.POINTER(_MCMCResult), vp]
    lib.mlmc_mimc.argtypes = [vp, ctypes.POINTER(_MIMCConfig), ctypes.POINTER(_MIMCResult), vp]
    lib.mlmc_estimate_resumable.argtypes = [vp, dbl, i32, ctypes.POINTER(ctypes.c_int), ctypes.c_int, i32,
                                            ctypes.POINTER(_EstimateState), i32, ctypes.POINTER(_EstimateState),
                                            ctypes.POINTER(_Result), vp]
    lib.mlmc_profile.argtypes = [vp, i32]
    lib.mlmc_profile_read.argtypes = [vp, i32, i32, ctypes.POINTER(dbl), ctypes.POINTER(i64),
                                      ctypes.POINTER(i64)]
    _lib = lib
    return lib


@dataclasses.dataclass
class Config:
    n0: int = 16
    m: int = 2
    L_max: int = 4
    K: int = 64
    sigma2: float = 1.0
    corr_len: float = 0.3
    f: float = 1.0
    k_p: float = 0.05
    alpha: float = 2.0
    beta: float = 4.0
    gamma: float = 4.0
    ir_max_iter: int = 10
    minres_max_iter: int = 5000
    seed: int = 1
    field: int = 0        # 0: exponential-covariance KL; 1: trigonometric field of sec. 5.1
    field_q: float = 2.0  # decay exponent q of the trigonometric field
    disc: int = 0         # 0: finite volumes (harmonic faces); 1: P1 elements on right triangles
    std_eps: float = 0.0  # standard MLMC with an iterative solver: fixed tolerance (0: 1e-6)


def _ptr(t):
    return None if t is None else ctypes.c_void_p(t.data_ptr())


def _stream():
    return ctypes.c_void_p(torch.cuda.current_stream().cuda_stream)


class MLMC:
    """A library context: KL bases of every level live on the current device."""

    def __init__(self, cfg: Config, device="cuda"):
        if not torch.cuda.is_available():
            raise MLMCError("no GPU visible: the MLMC library has no CPU path")
        self.lib = load_library()
        self.cfg = cfg
        self.device = torch.device(device)
        c = _Config(**dataclasses.asdict(cfg))
        h = ctypes.c_void_p()
        with torch.cuda.device(self.device):
            rc = self.lib.mlmc_create(ctypes.byref(c), ctypes.byref(h))
        if rc != 0:
            raise MLMCError("mlmc_create failed (%d)" % rc)
        self.h = h
        self._ws = None

    def close(self):
        if getattr(self, "h", None):
            self.lib.mlmc_destroy(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    # -------------------------------------------------------------- helpers
    def _check(self, rc, what):
        if rc < 0:
            msg = self.lib.mlmc_last_error(self.h)
            raise MLMCError("%s failed (%d): %s" % (what, rc, msg.decode() if msg else ""))
        return rc

    def _workspace(self, nbytes):
        if self._ws is None or self._ws.numel() < nbytes:
            self._ws = None
            torch.cuda.empty_cache()
            self._ws = torch.empty(max(nbytes, 256), dtype=torch.uint8, device=self.device)
        return self._ws

    @staticmethod
    def _opts(dtype="f64", solver="direct", eps_fine=0.0, eps_coarse=0.0, promote=True):
        return _LevelOpts(DTYPES[dtype], SOLVERS[solver], float(eps_fine), float(eps_coarse),
                          1 if promote else 0)

    def level_cells(self, level):
        return self.lib.mlmc_level_cells(self.h, level)

    def accuracy_targets(self, L):
        out = (ctypes.c_double * (L + 1))()
        self._check(self.lib.mlmc_accuracy_targets(self.h, L, out), "accuracy_targets")
        return list(out)

    def kl_basis(self, level):
        """Phi_level^T as a [K, (n+1)^2] float64 device tensor (a copy)."""
        n = self.level_cells(level)
        out = torch.empty((self.cfg.K, (n + 1) ** 2), dtype=torch.float64, device=self.device)
        self._check(self.lib.mlmc_get_kl_basis(self.h, level, _ptr(out), _stream()), "get_kl_basis")
        return out

    def workspace_bytes(self, level, n, **opt):
        o = self._opts(**opt)
        return self.lib.mlmc_workspace_bytes(self.h, level, n, ctypes.byref(o))

    KINDS = {"field": 0, "assembly": 1, "factor": 2, "solve": 3, "residual": 4, "minres": 5,
             "promote_factor": 6, "promote_solve": 7}

    def profile(self, enable=True):
        self._check(self.lib.mlmc_profile(self.h, 1 if enable else 0), "profile")

    def profile_read(self, kind, n):
        ms, cnt, smp = ctypes.c_double(), ctypes.c_int64(), ctypes.c_int64()
        self._check(self.lib.mlmc_profile_read(self.h, self.KINDS[kind], n, ctypes.byref(ms),
                                               ctypes.byref(cnt), ctypes.byref(smp)), "profile_read")
        return dict(ms=ms.value, launches=cnt.value, samples=smp.value)

    # -------------------------------------------------------------- entry points
    def fill_xi(self, level, first, n, out=None):
        """xi[n, K] of samples first .. first+n-1 of `level` (into `out` if given)."""
        xi = out if out is not None else torch.empty((n, self.cfg.K), dtype=torch.float64,
                                                      device=self.device)
        self._check(self.lib.mlmc_fill_xi(self.h, level, first, n, _ptr(xi), _stream()), "fill_xi")
        return xi

    def set_seed(self, seed):
        self._check(self.lib.mlmc_set_seed(self.h, int(seed) & 0xFFFFFFFFFFFFFFFF), "set_seed")
        self.cfg.seed = int(seed)

    def solve(self, level, xi, dtype="f64", solver="direct", eps=0.0, promote=True, want_u=False,
              own_workspace=False):
        """Batched solve on one grid.  own_workspace: solve in a workspace of
        this call's own (returned as out["ws"]) instead of the context's
        shared one, so that a later grad() can reuse its factor."""
        xi = xi.to(device=self.device, dtype=torch.float64).contiguous()
        S = xi.shape[0]
        n = self.level_cells(level)
        o = self._opts(dtype, solver, eps, 0.0, promote)
        nb = self.lib.mlmc_workspace_bytes(self.h, level, S, ctypes.byref(o))
        ws = (torch.empty(max(nb, 256), dtype=torch.uint8, device=self.device) if own_workspace
              else self._workspace(nb))
        q = torch.empty(S, dtype=torch.float64, device=self.device)
        u = torch.empty((S, (n - 1) ** 2), dtype=torch.float64, device=self.device) if want_u else None
        st = torch.empty(S, dtype=torch.uint8, device=self.device)
        it = torch.empty(S, dtype=torch.int32, device=self.device)
        rc = self._check(self.lib.mlmc_solve(self.h, level, S, _ptr(xi), ctypes.byref(o), _ptr(ws),
                                             ws.numel(), _ptr(q), _ptr(u), _ptr(st), _ptr(it),
                                             _stream()), "solve")
        out = dict(q=q, status=st, iters=it, rc=rc)
        if want_u:
            out["u"] = u
        if own_workspace:
            out["ws"] = ws
        return out

    def sample_level(self, level, xi, dtype="f64", solver="direct", eps_fine=0.0, eps_coarse=0.0,
                     promote=True, stats=True):
        xi = xi.to(device=self.device, dtype=torch.float64).contiguous()
        S = xi.shape[0]
        o = self._opts(dtype, solver, eps_fine, eps_coarse, promote)
        nb = self.lib.mlmc_workspace_bytes(self.h, level, S, ctypes.byref(o))
        ws = self._workspace(nb)
        qf = torch.empty(S, dtype=torch.float64, device=self.device)
        qc = torch.empty(S, dtype=torch.float64, device=self.device) if level > 0 else None
        y = torch.empty(S, dtype=torch.float64, device=self.device)
        st = torch.empty(S, dtype=torch.uint8, device=self.device)
        sts = _LevelStats()
        rc = self._check(self.lib.mlmc_sample_level(self.h, level, S, _ptr(xi), ctypes.byref(o),
                                                    _ptr(ws), ws.numel(), _ptr(qf), _ptr(qc),
                                                    _ptr(y), _ptr(st),
                                                    ctypes.byref(sts) if stats else None,
                                                    _stream()), "sample_level")
        out = dict(qf=qf, qc=qc, y=y, status=st, rc=rc)
        if stats:
            out["stats"] = {k: getattr(sts, k) for k, _ in _LevelStats._fields_}
        return out

    def sample_level_noalloc(self, level, xi, dtype="f64", solver="direct", eps_fine=0.0,
                             eps_coarse=0.0, promote=True, stats=True, out=None):
        """sample_level on the library's fixed per-device scratch (no workspace
        allocation by the library).  out: optional dict of preallocated
        output tensors qf, qc, y, status (else they are allocated here)."""
        xi = xi.to(device=self.device, dtype=torch.float64).contiguous()
        S = xi.shape[0]
        o = self._opts(dtype, solver, eps_fine, eps_coarse, promote)
        if out is None:
            out = dict(qf=torch.empty(S, dtype=torch.float64, device=self.device),
                       qc=torch.empty(S, dtype=torch.float64, device=self.device) if level > 0 else None,
                       y=torch.empty(S, dtype=torch.float64, device=self.device),
                       status=torch.empty(S, dtype=torch.uint8, device=self.device))
        sts = _LevelStats()
        rc = self._check(self.lib.mlmc_sample_level_noalloc(
            self.h, level, S, _ptr(xi), ctypes.byref(o), _ptr(out["qf"]), _ptr(out.get("qc")),
            _ptr(out["y"]), _ptr(out["status"]), ctypes.byref(sts) if stats else None, _stream()),
            "sample_level_noalloc")
        res = dict(out, rc=rc)
        if stats:
            res["stats"] = {k: getattr(sts, k) for k, _ in _LevelStats._fields_}
        return res

    def plan_levels(self, levels, xis, opts, use_graph=True):
        """A LevelPlan: opts is a list of dicts (dtype, solver, eps_fine, eps_coarse, promote)."""
        return LevelPlan(self, levels, xis, opts, use_graph)

    def autotune(self, level, xi, dtype="f32", solver="direct_ir", eps_fine=1e-6, eps_coarse=1e-6):
        xi = xi.to(device=self.device, dtype=torch.float64).contiguous()
        o = self._opts(dtype, solver, eps_fine, eps_coarse, True)
        nb = self.lib.mlmc_workspace_bytes(self.h, level, xi.shape[0], ctypes.byref(o))
        ws = self._workspace(nb)
        ch = (ctypes.c_int32 * 2)()
        self._check(self.lib.mlmc_autotune(self.h, level, xi.shape[0], _ptr(xi), ctypes.byref(o),
                                           _ptr(ws), ws.numel(), ch, _stream()), "autotune")
        return list(ch)

    def estimate(self, tol, n_init=1000, dtypes=None, solver="direct_ir", mixed=True, resume=None,
                 max_rounds=0):
        """Algorithm 4.1 (mlmc_estimate_resumable).  resume: a state dict of an
        earlier call (result["state"]) to continue from; max_rounds > 0 stops
        after that many rounds (rc == 2, MLMC_PAUSED, when not finished).  The
        returned "state" is JSON-serialisable."""
        L1 = self.cfg.L_max + 1
        dts = (ctypes.c_int * L1)(*[DTYPES[d] for d in (dtypes or ["f32"] * L1)])
        r = _Result()
        st_out = _EstimateState()
        st_in = _state_from_dict(resume) if resume is not None else None
        rc = self._check(self.lib.mlmc_estimate_resumable(
            self.h, float(tol), int(n_init), dts, SOLVERS[solver], 1 if mixed else 0,
            ctypes.byref(st_in) if st_in is not None else None, int(max_rounds), ctypes.byref(st_out),
            ctypes.byref(r), _stream()), "estimate")
        L = r.L
        return dict(estimate=r.estimate, var_est=r.var_est, L=L, converged=bool(r.converged),
                    N=list(r.N[:L + 1]), Yhat=list(r.Yhat[:L + 1]), s2=list(r.s2[:L + 1]),
                    C=list(r.C[:L + 1]), eps=list(r.eps[:L + 1]), wall_s=r.wall_s,
                    gpu_ms=r.gpu_ms, n_promoted=list(r.n_promoted[:L1]),
                    n_noconv=list(r.n_noconv[:L1]), rc=rc, state=_state_to_dict(st_out))

    def mcmc(self, L, chains, steps, obs, noise_sd, burn_in=10, subsample=2, pcn_beta=0.5, opts=None,
             seed=None):
        """Multilevel MCMC (mlmc_mcmc): obs is a list of (x, y, value) at interior
        nodes of the coarsest grid, steps a list of recorded steps per level,
        opts a list of per-level option dicts (dtype, solver, eps_fine, eps_coarse)."""
        c = _MCMCConfig()
        c.L, c.chains, c.burn_in, c.subsample = int(L), int(chains), int(burn_in), int(subsample)
        for l, k in enumerate(steps):
            c.steps[l] = int(k)
        c.pcn_beta, c.noise_sd, c.n_obs = float(pcn_beta), float(noise_sd), len(obs)
        for j, (x, y, v) in enumerate(obs):
            c.obs_x[j], c.obs_y[j], c.obs_value[j] = x, y, v
        for l in range(L + 1):
            o = (opts or [{}] * (L + 1))[l]
            c.opts[l] = self._opts(**o)
        c.seed = int(self.cfg.seed if seed is None else seed) & 0xFFFFFFFFFFFFFFFF
        r = _MCMCResult()
        rc = self._check(self.lib.mlmc_mcmc(self.h, ctypes.byref(c), ctypes.byref(r), _stream()), "mcmc")
        return dict(estimate=r.estimate, Yhat=list(r.Yhat[:L + 1]), var_mean=list(r.var_mean[:L + 1]),
                    accept=list(r.accept[:L + 1]), accept_coarse=list(r.accept_coarse[:L + 1]),
                    solves=r.solves, wall_s=r.wall_s, rc=rc)

    def mimc(self, indices, N, K0, opts=None, seed=None):
        """Multi-index Monte Carlo (mlmc_mimc): indices a list of (l, k) (grid
        index, truncation index: the first K0 * 2**k modes), N the samples per
        index, opts a list of per-index option dicts (dtype, solver, eps_fine,
        eps_coarse).  Returns the estimate and the per-index means, variances,
        promotion and non-convergence counts."""
        c = _MIMCConfig()
        c.n_idx, c.K0 = len(indices), int(K0)
        for i, (l, k) in enumerate(indices):
            c.idx_l[i], c.idx_k[i], c.N[i] = int(l), int(k), int(N[i])
            c.opts[i] = self._opts(**((opts or [{}] * len(indices))[i]))
        c.seed = int(self.cfg.seed if seed is None else seed) & 0xFFFFFFFFFFFFFFFF
        r = _MIMCResult()
        rc = self._check(self.lib.mlmc_mimc(self.h, ctypes.byref(c), ctypes.byref(r), _stream()), "mimc")
        n = len(indices)
        return dict(estimate=r.estimate, var_estimate=r.var_estimate, mean=list(r.mean[:n]), var=list(r.var[:n]),
                    n_promoted=list(r.n_promoted[:n]), n_noconv=list(r.n_noconv[:n]), solves=r.solves,
                    wall_s=r.wall_s, rc=rc)

    def grad_from(self, level, xi, ws, grad_q=None, eps_adjoint=1e-10, dtype="f32",
                  solver="direct_ir", eps=1e-10):
        """grad_q[s] * dQ/dxi[s, :] for the samples of a preceding solve() on
        workspace ws with the same level, xi and options (its factor and
        solution are reused by the adjoint)."""
        xi = xi.to(device=self.device, dtype=torch.float64).contiguous()
        S = xi.shape[0]
        o = self._opts(dtype, solver, eps, 0.0, True)
        g = torch.empty((S, self.cfg.K), dtype=torch.float64, device=self.device)
        gq = None if grad_q is None else grad_q.to(device=self.device, dtype=torch.float64).contiguous()
        self._check(self.lib.mlmc_grad(self.h, level, S, _ptr(xi), _ptr(gq), ctypes.byref(o),
                                       float(eps_adjoint), _ptr(ws), ws.numel(), _ptr(g), _stream()),
                    "grad")
        return g

    def grad(self, level, xi, grad_q=None, eps_adjoint=1e-10, dtype="f32", solver="direct_ir",
             eps=1e-10):
        """(Q, dQ/dxi * grad_q): forward solve, then the adjoint on the same workspace."""
        xi = xi.to(device=self.device, dtype=torch.float64).contiguous()
        fw = self.solve(level, xi, dtype=dtype, solver=solver, eps=eps, promote=True)
        g = self.grad_from(level, xi, self._ws, grad_q, eps_adjoint, dtype, solver, eps)
        return fw["q"], g


class LevelPlan:
    """Persistent buffers for repeated mlmc_sample_levels calls on fixed inputs.

    levels, xis (device tensors [N_l, K]) and per-level options are fixed at
    construction; run() launches every level concurrently (optionally as one
    replayed HIP graph) and returns the Y tensors.
    """

    def __init__(self, ctx, levels, xis, opts, use_graph=True):
        self.ctx, self.use_graph = ctx, use_graph
        self.levels = list(levels)
        self.xis = [x.to(device=ctx.device, dtype=torch.float64).contiguous() for x in xis]
        L = len(self.levels)
        self.c_levels = (ctypes.c_int32 * L)(*self.levels)
        self.c_n = (ctypes.c_int64 * L)(*[x.shape[0] for x in self.xis])
        self.c_xi = (ctypes.c_void_p * L)(*[x.data_ptr() for x in self.xis])
        self.c_opts = (_LevelOpts * L)(*[MLMC._opts(**o) for o in opts])
        nb = ctx.lib.mlmc_levels_workspace_bytes(ctx.h, L, self.c_levels, self.c_n, self.c_opts)
        if nb == 0:
            raise MLMCError("bad level plan")
        self.ws = torch.empty(nb, dtype=torch.uint8, device=ctx.device)
        self.y = [torch.empty(x.shape[0], dtype=torch.float64, device=ctx.device) for x in self.xis]
        self.c_y = (ctypes.c_void_p * L)(*[y.data_ptr() for y in self.y])

    def run(self, stats=False):
        L = len(self.levels)
        st = (_LevelStats * L)() if stats else None
        rc = self.ctx._check(self.ctx.lib.mlmc_sample_levels(
            self.ctx.h, L, self.c_levels, self.c_n, self.c_xi, self.c_opts, _ptr(self.ws),
            self.ws.numel(), self.c_y, st, 1 if self.use_graph else 0, _stream()), "sample_levels")
        out = dict(y=self.y, rc=rc)
        if stats:
            out["stats"] = [{k: getattr(x, k) for k, _ in _LevelStats._fields_} for x in st]
        return out


class MLMCQoI(torch.autograd.Function):
    """Q_l(xi) on one grid with the adjoint gradient as backward.

    forward(ctx_obj, level, xi, dtype, eps) -> Q[S] solves only, in a
    workspace of its own that keeps the factor and the solution; backward
    runs the library's adjoint on that workspace with grad_q = grad_out and
    returns grad_q[s] * dQ/dxi[s, :].  The workspace is released with the
    autograd graph (after backward, or when no backward follows).
    """

    @staticmethod
    def forward(ctx, lib_ctx, level, xi, dtype="f32", eps=1e-10):
        solver = "direct_ir" if dtype != "f64" else "direct"
        xd = xi.detach().to(device=lib_ctx.device, dtype=torch.float64).contiguous()
        fw = lib_ctx.solve(level, xd, dtype=dtype, solver=solver, eps=eps, promote=True,
                           own_workspace=True)
        ctx.lib_ctx, ctx.level, ctx.dtype, ctx.solver, ctx.eps = lib_ctx, level, dtype, solver, eps
        ctx.ws, ctx.xi = fw["ws"], xd
        return fw["q"].to(xi.dtype)

    @staticmethod
    def backward(ctx, grad_out):
        g = ctx.lib_ctx.grad_from(ctx.level, ctx.xi, ctx.ws, grad_out, eps_adjoint=ctx.eps,
                                  dtype=ctx.dtype, solver=ctx.solver, eps=ctx.eps)
        ctx.ws = None
        return None, None, g, None, None
