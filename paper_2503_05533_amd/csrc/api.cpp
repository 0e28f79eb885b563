// Host side of libmlmc: context, KL set-up, workspace layout, the per-grid
// solve driver (factorisation, Algorithm 2.1 refinement, promotion, MINRES),
// the MLMC level pairing, the Algorithm 4.1 driver and the adjoint gradient.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <chrono>
#include <cmath>
#include <cstdarg>
#include <cstdio>
#include <cstring>
#include <functional>
#include <string>
#include <vector>

#include "../../include/mlmc.h"
#include "kernels.h"

using namespace mlmc;

struct mlmc_ctx {
    mlmc_config cfg;
    int device = 0;
    std::vector<double *> phit;  // per level: [K][(n+1)^2] FP64 on the device
    std::string err;
    int *d_counter = nullptr;    // device scratch: active-sample counters
    double *d_sums = nullptr;    // device scratch: level sums (16 doubles)
    int *h_counter = nullptr;    // pinned host mirror
    double *h_sums = nullptr;
    hipEvent_t ev0 = nullptr, ev1 = nullptr;
    // kernel timing records (mlmc_profile)
    struct prof_rec { int kind, n; int64_t samples; hipEvent_t a, b; };
    bool prof_on = false;
    std::vector<prof_rec> prof;
    std::vector<hipEvent_t> ev_pool;
    // refinement-kernel variant per (factor dtype, log2 n), 0 = built-in default
    int ir_variant[5][9] = {};
    // factorisation variant per (factor dtype, log2 n): 0 default, 1 FP32 MFMA
    // products for the FP16/BF16 factors (autotuner)
    int factor_variant[5][9] = {};
    // concurrent multi-level launches: two streams per level, events, cached graph
    std::vector<hipStream_t> lstreams;
    std::vector<hipEvent_t> levents;
    hipStream_t cap_stream = nullptr;
    // eager multi-level launches: one stream per hardware queue, events
    std::vector<hipStream_t> qstreams;
    std::vector<hipEvent_t> qevents;
    // mlmc_estimate's workspace (chunk workspaces and xi buffers), kept
    void *est_buf = nullptr;
    size_t est_bytes = 0;
    hipGraph_t graph = nullptr;
    hipGraphExec_t graph_exec = nullptr;
    std::vector<uintptr_t> graph_key;
    bool capturing = false;
    // device address of the library's fixed scratch array on this device
    // (mlmc_sample_level_noalloc), taken at mlmc_create
    void *scratch = nullptr;
};

namespace {

int fail(mlmc_ctx *c, int code, const char *fmt, ...)
{
    if (c) {
        char buf[512];
        va_list ap;
        va_start(ap, fmt);
        vsnprintf(buf, sizeof buf, fmt, ap);
        va_end(ap);
        c->err = buf;
    }
    return code;
}

#define HIPCHK(expr)                                                                       \
    do {                                                                                   \
        hipError_t e_ = (expr);                                                            \
        if (e_ != hipSuccess)                                                              \
            return fail(ctx, MLMC_EHIP, "%s: %s (%s:%d)", #expr, hipGetErrorString(e_),    \
                        __FILE__, __LINE__);                                               \
    } while (0)

#define PROF(kind, n_, cnt_, expr)                                                         \
    do {                                                                                   \
        prof_scope ps_(ctx, kind, n_, cnt_, st);                                           \
        HIPCHK(expr);                                                                      \
    } while (0)

inline size_t align256(size_t b) { return (b + 255) & ~(size_t)255; }
// A caller pointer is usable when it is NULL (optional buffers) or aligned to
// its element size.
inline bool aligned(const void *p, size_t a) { return ((uintptr_t)p & (a - 1)) == 0; }
inline size_t dtype_bytes(int dt) { return dt == MLMC_F64 ? 8 : (dt == MLMC_F32 ? 4 : (dt == MLMC_FP8 ? 1 : 2)); }
inline bool is_pow2(int v) { return v > 0 && (v & (v - 1)) == 0; }
inline bool is_minres(int solver) { return solver == MLMC_MINRES || solver == MLMC_MINRES_IR; }
// solvers without a factorisation
inline bool is_iterative(int solver) { return is_minres(solver) || solver == MLMC_MGCG; }
inline int ilog2(int v) { int l = 0; while ((1 << (l + 1)) <= v) ++l; return l; }

// ---------------------------------------------------------------- kernel timing

hipEvent_t pool_event(mlmc_ctx *c)
{
    if (!c->ev_pool.empty()) {
        hipEvent_t e = c->ev_pool.back();
        c->ev_pool.pop_back();
        return e;
    }
    hipEvent_t e = nullptr;
    if (hipEventCreate(&e) != hipSuccess) return nullptr;
    return e;
}

// Bracket one launch with events when profiling is on.
struct prof_scope {
    mlmc_ctx *c;
    hipStream_t st;
    int kind, n;
    int64_t samples;
    hipEvent_t a = nullptr;
    prof_scope(mlmc_ctx *c_, int kind_, int n_, int64_t s_, hipStream_t st_)
        : c(c_), st(st_), kind(kind_), n(n_), samples(s_)
    {
        if (c->prof_on && !c->capturing && (a = pool_event(c))) (void)hipEventRecord(a, st);
    }
    ~prof_scope()
    {
        if (!a) return;
        hipEvent_t b = pool_event(c);
        if (!b) return;
        (void)hipEventRecord(b, st);
        c->prof.push_back({kind, n, samples, a, b});
    }
};

// ---------------------------------------------------------------- KL set-up
// Separable exponential covariance sigma^2 exp(-|x1-y1|/lam) exp(-|x2-y2|/lam).
// 1D eigenvalues mu = 2 lam / (1 + lam^2 w^2) where w solves
// (lam^2 w^2 - 1) sin w = 2 lam w cos w, one root per ((k-1) pi, k pi);
// eigenfunctions (sin w x + lam w cos w x) / ||.||.

double kl_eq(double w, double lam) { return (lam * lam * w * w - 1.0) * std::sin(w) - 2.0 * lam * w * std::cos(w); }

// Illinois (modified regula falsi) on a sign-changing bracket.
double kl_root(int k, double lam)
{
    const double pi = 3.14159265358979323846;
    double lo = (k - 1) * pi, hi = k * pi;
    double flo = k == 1 ? -1.0 : kl_eq(lo, lam), fhi = kl_eq(hi, lam);
    if (k == 1) lo = 0.0;
    int side = 0;
    for (int it = 0; it < 300 && hi - lo > 4e-16 * hi; ++it) {
        double w = (lo * fhi - hi * flo) / (fhi - flo);
        if (!(w > lo && w < hi)) w = 0.5 * (lo + hi);
        const double fw = kl_eq(w, lam);
        if (fw == 0.0) return w;
        if ((fw < 0) == (flo < 0)) {
            lo = w;
            flo = fw;
            if (side == -1) fhi *= 0.5;
            side = -1;
        } else {
            hi = w;
            fhi = fw;
            if (side == 1) flo *= 0.5;
            side = 1;
        }
    }
    return 0.5 * (lo + hi);
}

struct kl_mode { double prod; int i, j; };

// Trigonometric field of Sec. 5.1 (eq. of the random coefficient):
// Phi[p, j-1] = sigma j^-q sin(2 pi j x) cos(2 pi j y), j = 1..K.
void build_phit_trig(const mlmc_config &c, std::vector<std::vector<double>> &out)
{
    const double pi = 3.14159265358979323846, sigma = std::sqrt(c.sigma2);
    out.assign(c.L_max + 1, {});
    for (int l = 0; l <= c.L_max; ++l) {
        const int n = c.n0 << l, P = (n + 1) * (n + 1);
        std::vector<double> &ph = out[l];
        ph.assign((size_t)c.K * P, 0.0);
        for (int k = 0; k < c.K; ++k) {
            const double jj = k + 1.0, amp = sigma * std::pow(jj, -c.field_q);
            for (int iy = 0; iy <= n; ++iy) {
                const double cy = std::cos(2.0 * pi * jj * iy / n);
                for (int ix = 0; ix <= n; ++ix)
                    ph[(size_t)k * P + iy * (n + 1) + ix] = amp * std::sin(2.0 * pi * jj * ix / n) * cy;
            }
        }
    }
}

int build_phit(mlmc_ctx *ctx, std::vector<std::vector<double>> &out)
{
    const mlmc_config &c = ctx->cfg;
    if (c.field == 1) {
        build_phit_trig(c, out);
        return MLMC_OK;
    }
    const double lam = c.corr_len;
    int R = 64;
    std::vector<double> w, mu, nu;
    std::vector<kl_mode> sel;
    for (;;) {
        w.resize(R);
        mu.resize(R);
        nu.resize(R);
        for (int k = 0; k < R; ++k) {
            w[k] = kl_root(k + 1, lam);
            mu[k] = 2.0 * lam / (1.0 + lam * lam * w[k] * w[k]);
            const double s2 = std::sin(2.0 * w[k]), c2 = std::cos(2.0 * w[k]);
            nu[k] = 0.5 - s2 / (4.0 * w[k]) + lam * lam * w[k] * w[k] * (0.5 + s2 / (4.0 * w[k])) +
                    0.5 * lam * (1.0 - c2);
        }
        std::vector<kl_mode> all;
        all.reserve((size_t)R * R);
        for (int i = 0; i < R; ++i)
            for (int j = 0; j < R; ++j) all.push_back({mu[i] * mu[j], i, j});
        std::sort(all.begin(), all.end(), [](const kl_mode &a, const kl_mode &b) {
            if (a.prod != b.prod) return a.prod > b.prod;
            if (a.i != b.i) return a.i < b.i;
            return a.j < b.j;
        });
        sel.assign(all.begin(), all.begin() + c.K);
        // every pair touching an index >= R has product <= mu_0 mu_{R-1}
        if (mu[0] * mu[R - 1] < sel.back().prod) break;
        R *= 2;
        if (R > 4096) return fail(ctx, MLMC_EINVAL, "KL: too many modes requested");
    }
    const double sigma = std::sqrt(c.sigma2);
    out.assign(c.L_max + 1, {});
    for (int l = 0; l <= c.L_max; ++l) {
        const int n = c.n0 << l, P = (n + 1) * (n + 1);
        std::vector<double> f1((size_t)R * (n + 1));  // phi_r(t/n)
        for (int r = 0; r < R; ++r) {
            const double inv = 1.0 / std::sqrt(nu[r]);
            for (int t = 0; t <= n; ++t) {
                const double x = (double)t / n;
                f1[(size_t)r * (n + 1) + t] = (std::sin(w[r] * x) + lam * w[r] * std::cos(w[r] * x)) * inv;
            }
        }
        std::vector<double> &ph = out[l];
        ph.assign((size_t)c.K * P, 0.0);
        for (int k = 0; k < c.K; ++k) {
            const int i = sel[k].i, j = sel[k].j;
            const double amp = sigma * std::sqrt(mu[i] * mu[j]);
            for (int iy = 0; iy <= n; ++iy)
                for (int ix = 0; ix <= n; ++ix)
                    ph[(size_t)k * P + iy * (n + 1) + ix] =
                        amp * f1[(size_t)i * (n + 1) + ix] * f1[(size_t)j * (n + 1) + iy];
        }
    }
    return MLMC_OK;
}

// ---------------------------------------------------------------- workspace

struct grid_layout {
    int n, m, M;
    int64_t S;
    size_t vec;  // padded vector length per sample
    size_t off_a, off_sc, off_gam, off_beta, off_x, off_r, off_z, off_lam, off_gz;
    size_t off_factor, off_promo, off_state, off_relres, off_q, off_iters, off_idx;
    size_t off_mr;  // MINRES vectors (7 per sample, FP64 or FP32)
    size_t off_mgv, off_mgh;  // multigrid CG: 5 FP64 node vectors, the FP32 hierarchy
    size_t off_cnt; // device counters (promotion)
    int64_t promo_slots;
    size_t bytes;
};

grid_layout make_layout(int n, int64_t S, const mlmc_level_opts &o)
{
    grid_layout L{};
    L.n = n;
    L.m = n - 1;
    L.M = n;
    L.S = S;
    L.vec = (size_t)L.m * L.M;
    const size_t vb = align256(S * L.vec * 8);
    size_t off = 0;
    auto take = [&](size_t b) { size_t o2 = off; off += align256(b); return o2; };
    L.off_a = take(S * (size_t)(n + 1) * (n + 1) * 8);
    L.off_gz = take(S * (size_t)(n + 1) * (n + 1) * 8);
    L.off_sc = take(vb);
    L.off_gam = take(vb);
    L.off_beta = take(vb);
    L.off_x = take(vb);
    L.off_r = take(vb);
    L.off_z = take(vb);
    L.off_lam = take(vb);
    const bool direct = !is_iterative(o.solver);
    const int dt = o.solver == MLMC_DIRECT ? MLMC_F64 : o.factor_dtype;
    L.off_factor = take(direct ? S * factor_entries_per_sample(dt, n) * dtype_bytes(dt) : 0);
    // every sample can be re-solved with an FP64 factor without a host round trip
    L.promo_slots = (direct && dt != MLMC_F64 && o.promote) ? S : 0;
    L.off_promo = take(L.promo_slots * factor_entries_per_sample(MLMC_F64, n) * 8);
    // 7 FP64 vectors per sample: also room for the FP64 re-solve of MINRES-IR samples
    L.off_mr = take(is_minres(o.solver) ? 7 * S * L.vec * 8 : 0);
    const bool mg = o.solver == MLMC_MGCG;
    L.off_mgv = take(mg ? 5 * S * (size_t)(n + 1) * (n + 1) * 8 : 0);
    L.off_mgh = take(mg ? S * mgcg_floats_per_sample(n) * 4 : 0);
    L.off_state = take(S * 4);
    L.off_relres = take(S * 8);
    L.off_q = take(S * 8);
    L.off_iters = take(S * 4);
    L.off_idx = take(S * 4);
    L.off_cnt = take(64);
    L.bytes = off;
    return L;
}

struct level_layout {
    grid_layout fine, coarse;
    size_t off_fine, off_coarse, off_qf, off_qc, off_y, off_sums, bytes;
};

level_layout make_level_layout(const mlmc_config &c, int level, int64_t S, const mlmc_level_opts &o)
{
    level_layout L{};
    const int nf = c.n0 << level;
    L.fine = make_layout(nf, S, o);
    size_t off = 0;
    L.off_fine = off;
    off += align256(L.fine.bytes);
    if (level > 0) {
        L.coarse = make_layout(nf / 2, S, o);
        L.off_coarse = off;
        off += align256(L.coarse.bytes);
    }
    L.off_qf = off;
    off += align256(S * 8);
    L.off_qc = off;
    off += align256(S * 8);
    L.off_y = off;
    off += align256(S * 8);
    L.off_sums = off;
    off += 256;
    L.bytes = off;
    return L;
}

template <typename T> T *at(void *base, size_t off) { return (T *)((char *)base + off); }

int check_level(mlmc_ctx *ctx, int level)
{
    if (!ctx) return MLMC_EINVAL;
    if (level < 0 || level > ctx->cfg.L_max) return fail(ctx, MLMC_EINVAL, "level %d out of range", level);
    return MLMC_OK;
}

// Options of a call on level `level`: the fine grid, and with `pair` also
// the coarse partner (level - 1), must offer the factor dtype.
int check_opts(mlmc_ctx *ctx, const mlmc_level_opts *o, int level, bool pair)
{
    if (!o) return fail(ctx, MLMC_EINVAL, "opts is NULL");
    if (o->factor_dtype < MLMC_F64 || o->factor_dtype > MLMC_FP8)
        return fail(ctx, MLMC_EINVAL, "bad factor dtype");
    if (o->solver < MLMC_DIRECT || o->solver > MLMC_MGCG) return fail(ctx, MLMC_EINVAL, "bad solver");
    if (!(o->eps_fine >= 0.0) || !(o->eps_coarse >= 0.0)) return fail(ctx, MLMC_EINVAL, "bad eps");
    if (o->solver == MLMC_DIRECT_IR) {
        const int n = ctx->cfg.n0 << level;
        if (!dtype_on_grid(o->factor_dtype, n) || (pair && level > 0 && !dtype_on_grid(o->factor_dtype, n / 2)))
            return fail(ctx, MLMC_ENOTIMPL, "factor dtype %d is not available on the %d-cell grid", o->factor_dtype,
                        n);
    }
    return MLMC_OK;
}

// Initial solve + Algorithm 2.1 on the stored factor for all samples of a
// grid (solution into x, rhs h^2 fconst), then, for a low-precision factor,
// device-side compaction of the samples that did not converge and a second
// pass with an FP64 factor for them.  Asynchronous on `st`.
int refine(mlmc_ctx *ctx, const grid_layout &L, void *ws, int dt, bool direct, double fconst,
           double eps, double *x, double *q, int32_t *iters, hipStream_t st, bool fwd_done = false)
{
    const int n = L.n, S = (int)L.S;
    uint32_t *state = at<uint32_t>(ws, L.off_state);
    double *relres = at<double>(ws, L.off_relres);
    ir_args g{};
    g.n = n;
    g.nblocks = S;
    g.fconst = fconst;
    g.a = at<double>(ws, L.off_a);
    g.sc = at<double>(ws, L.off_sc);
    g.beta = at<double>(ws, L.off_beta);
    g.factor = at<void>(ws, L.off_factor);
    g.x = x;
    g.r = at<double>(ws, L.off_r);
    g.z = at<double>(ws, L.off_z);
    g.eps = eps;
    g.imax = direct ? 0 : ctx->cfg.ir_max_iter;
    g.direct = direct ? 1 : 0;
    g.state = state;
    g.relres = relres;
    g.q = q;
    g.iters = iters;
    g.variant = ctx->ir_variant[dt][ilog2(n)];
    // 2: the factorisation also ran the back sweep (x0 in x; block layouts)
    g.fwd_done = !fwd_done ? 0 : (n > 16 && factor_solves_initial(dt, n) ? 2 : 1);
    g.disc = ctx->cfg.disc;
    PROF(3, n, S, launch_ir(dt, g, st));
    if (L.promo_slots > 0 && dt != MLMC_F64) {
        int *idx = at<int>(ws, L.off_idx);
        int *cnt = at<int>(ws, L.off_cnt);
        const int np = (int)L.promo_slots;
        void *pf = at<void>(ws, L.off_promo);
        HIPCHK(launch_zero_int(cnt, 1, st));
        HIPCHK(launch_collect(S, state, idx, cnt, st));
        HIPCHK(launch_reset_subset(np, idx, cnt, state, relres, st));
        PROF(6, n, np, launch_factor(MLMC_F64, n, np, at<double>(ws, L.off_a), at<double>(ws, L.off_sc),
                                     at<double>(ws, L.off_beta), at<double>(ws, L.off_gam), pf, idx, cnt, 0,
                                     state, 0.0, nullptr, nullptr, ctx->cfg.disc, 0, st));
        ir_args p = g;
        p.nblocks = np;
        p.factor = pf;
        p.idx = idx;
        p.count = cnt;
        p.imax = ctx->cfg.ir_max_iter;
        p.direct = 0;
        p.variant = ctx->ir_variant[MLMC_F64][ilog2(n)];
        p.fwd_done = 0;
        PROF(7, n, np, launch_ir(MLMC_F64, p, st));
    }
    return MLMC_OK;
}

// Solve one batch on one grid, asynchronously on `st`: field GEMM, scaled
// coefficients, factorisation, then one per-sample kernel running the
// initial solve and the Algorithm 2.1 loop.  Samples that do not converge
// (promote != 0, low-precision factor) are compacted on the device and
// re-solved with an FP64 factor in a second pass, up to promo_slots of them.
// q (S doubles, device) receives Q; iters the corrections per sample.
// ev_main (optional) is recorded on st after the set-up kernels, before the
// factorisation (or the iterative solver).
int solve_grid(mlmc_ctx *ctx, const grid_layout &L, int level, const double *xi,
               const mlmc_level_opts &o, double eps, void *ws, double *q, int32_t *iters,
               hipStream_t st, hipEvent_t ev_main = nullptr)
{
    const int n = L.n, S = (int)L.S, K = ctx->cfg.K, P = (n + 1) * (n + 1);
    if (S == 0) return MLMC_OK;
    double *a = at<double>(ws, L.off_a);
    double *sc = at<double>(ws, L.off_sc), *gam = at<double>(ws, L.off_gam);
    double *beta = at<double>(ws, L.off_beta);
    uint32_t *state = at<uint32_t>(ws, L.off_state);
    double *relres = at<double>(ws, L.off_relres);
    PROF(0, n, S, launch_field(S, K, P, xi, ctx->phit[level], a, st));
    // the n = 16 factorisation forms the scaled operator itself
    if (o.solver == MLMC_MGCG) {
        HIPCHK(launch_init_state(S, state, relres, st));
        if (ev_main) HIPCHK(hipEventRecord(ev_main, st));
        PROF(5, n, S, launch_mgcg(n, S, ctx->cfg.f, a, at<double>(ws, L.off_x), at<double>(ws, L.off_mgv),
                                  at<float>(ws, L.off_mgh), eps, ctx->cfg.minres_max_iter, state, relres, q, iters,
                                  ctx->cfg.disc, st));
        return MLMC_OK;
    }
    if (is_minres(o.solver) || !factor_forms_coeffs(n)) PROF(1, n, S, launch_coeffs(n, S, a, sc, gam, beta, ctx->cfg.disc, st));
    HIPCHK(launch_init_state(S, state, relres, st));
    if (ev_main) HIPCHK(hipEventRecord(ev_main, st));
    if (is_minres(o.solver)) {
        // MINRES: FP64 vectors, a restart from the true residual at most 8
        // times; MINRES-IR: FP32 inner vectors, up to ir_max_iter refinements
        const bool low = o.solver == MLMC_MINRES_IR;
        PROF(5, n, S, launch_minres(n, S, ctx->cfg.f, a, sc, gam, beta, at<double>(ws, L.off_x),
                                    at<double>(ws, L.off_r), at<void>(ws, L.off_mr), low ? 1 : 0, eps,
                                    ctx->cfg.minres_max_iter, low ? ctx->cfg.ir_max_iter : 8, nullptr, nullptr,
                                    state, relres, q, iters, ctx->cfg.disc, st));
        if (low && o.promote) {
            // samples whose FP32-vector refinement did not converge: FP64 MINRES,
            // compacted on the device (workgroups beyond the count exit)
            int *idx = at<int>(ws, L.off_idx);
            int *cnt = at<int>(ws, L.off_cnt);
            HIPCHK(launch_zero_int(cnt, 1, st));
            HIPCHK(launch_collect(S, state, idx, cnt, st));
            HIPCHK(launch_reset_subset(S, idx, cnt, state, relres, st));
            PROF(5, n, S, launch_minres(n, S, ctx->cfg.f, a, sc, gam, beta, at<double>(ws, L.off_x),
                                        at<double>(ws, L.off_r), at<void>(ws, L.off_mr), 0, eps,
                                        ctx->cfg.minres_max_iter, 8, idx, cnt, state, relres, q, iters,
                                        ctx->cfg.disc, st));
        }
        return MLMC_OK;
    }
    const bool direct = o.solver == MLMC_DIRECT;
    const int dt = direct ? MLMC_F64 : o.factor_dtype;
    void *factor = at<void>(ws, L.off_factor);
    // the factorisation also runs the initial solve's forward sweep (rhs h^2 f),
    // at n = 16 the whole initial solve
    const bool fwd = factor_fuses_forward(dt, n);
    const double h = 1.0 / n;
    double *x = at<double>(ws, L.off_x);
    PROF(2, n, S, launch_factor(dt, n, S, a, sc, beta, gam, factor, nullptr, nullptr, 0, state, h * h * ctx->cfg.f,
                                fwd ? at<double>(ws, L.off_z) : nullptr,
                                fwd && factor_solves_initial(dt, n) ? x : nullptr, ctx->cfg.disc,
                                ctx->factor_variant[dt][ilog2(n)], st));
    return refine(ctx, L, ws, dt, direct, ctx->cfg.f, eps, x, q, iters, st, fwd);
}


// Enqueue one MLMC level: the fine grid on `sf`, the coarse grid on `sc`
// (which may equal sf), then the pairing and level sums on `sf` after the
// coarse grid (event `ev`).  Outputs default to workspace buffers.
int level_enqueue(mlmc_ctx *ctx, int level, int64_t n, const double *xi, const mlmc_level_opts &o,
                  void *ws_dev, const level_layout &LL, double *q_fine, double *q_coarse, double *y,
                  uint8_t *status, hipStream_t sf, hipStream_t scs, hipEvent_t ev)
{
    if (n == 0) return MLMC_OK;
    double *qf = q_fine ? q_fine : at<double>(ws_dev, LL.off_qf);
    double *qc = q_coarse ? q_coarse : at<double>(ws_dev, LL.off_qc);
    void *wf = at<void>(ws_dev, LL.off_fine);
    int rc = solve_grid(ctx, LL.fine, level, xi, o, o.eps_fine, wf, qf, at<int32_t>(wf, LL.fine.off_iters), sf);
    if (rc) return rc;
    const uint32_t *stc = nullptr;
    const int32_t *itc = nullptr;
    if (level > 0) {
        void *wc = at<void>(ws_dev, LL.off_coarse);
        rc = solve_grid(ctx, LL.coarse, level - 1, xi, o, o.eps_coarse, wc, qc,
                        at<int32_t>(wc, LL.coarse.off_iters), scs);
        if (rc) return rc;
        stc = at<uint32_t>(wc, LL.coarse.off_state);
        itc = at<int32_t>(wc, LL.coarse.off_iters);
        if (scs != sf) {
            HIPCHK(hipEventRecord(ev, scs));
            HIPCHK(hipStreamWaitEvent(sf, ev, 0));
        }
    }
    HIPCHK(launch_pair_sums((int)n, qf, level > 0 ? qc : nullptr, at<uint32_t>(wf, LL.fine.off_state), stc,
                            at<int32_t>(wf, LL.fine.off_iters), itc, y, status, at<double>(ws_dev, LL.off_sums),
                            sf));
    return MLMC_OK;
}


// Eager multi-level schedule.  The device runs a process's work on a few
// hardware queues (four by default) and every stream is bound to one of
// them, so two independent chains on streams that share a queue run one
// after the other.  The grids of all levels (fine and coarse) are therefore
// spread over exactly kQueues streams created back to back: the most
// expensive grid (the fine grid of the finest level, a latency-bound chain
// of factor and refinement) alone on the first, the others longest first
// onto the least loaded of the rest.  The other queues start only when the
// first grid's factorisation is next in its queue (an event after its
// set-up kernels): its workgroups then take their CUs before the other
// grids' kernels fill them, and run at the rate they have alone (started
// together, the other grids' workgroups held the LDS and registers that
// the factorisation's workgroups waited for, and the chain took 1.8x its
// time alone).  A level's pairing and sums are enqueued after all grids (so
// that no grid waits behind them), on the stream of its fine grid, after an
// event of its coarse grid.  Cost model: samples x n^3.5 (between the n^3 of
// the solves and the n^4 of the factorisation).
constexpr int kQueues = 4;

// The context's kQueues streams (created back to back, default priority) and
// at least nev events.
int ensure_queues(mlmc_ctx *ctx, size_t nev)
{
    while (ctx->qstreams.size() < (size_t)kQueues) {
        hipStream_t s2;
        HIPCHK(hipStreamCreateWithFlags(&s2, hipStreamNonBlocking));
        ctx->qstreams.push_back(s2);
    }
    while (ctx->qevents.size() < nev) {
        hipEvent_t e;
        HIPCHK(hipEventCreateWithFlags(&e, hipEventDisableTiming));
        ctx->qevents.push_back(e);
    }
    return MLMC_OK;
}

int enqueue_levels_queued(mlmc_ctx *ctx, int n_levels, const int32_t *levels, const int64_t *n,
                          const double *const *xi_dev, const mlmc_level_opts *opts, void *ws_dev,
                          const std::vector<level_layout> &LL, const std::vector<size_t> &off,
                          double *const *y_dev, hipStream_t os)
{
    if (int rc = ensure_queues(ctx, 2 + 2 * (size_t)n_levels + kQueues)) return rc;
    struct job { int li, coarse; double cost; };
    std::vector<job> jobs;
    for (int i = 0; i < n_levels; ++i) {
        if (n[i] == 0) continue;
        for (int c = 0; c < (levels[i] > 0 ? 2 : 1); ++c) {
            const double nn = (double)(ctx->cfg.n0 << (levels[i] - c));
            jobs.push_back({i, c, (double)n[i] * std::pow(nn, 3.5)});
        }
    }
    std::stable_sort(jobs.begin(), jobs.end(), [](const job &a, const job &b) { return a.cost > b.cost; });
    std::vector<int> qof(jobs.size());
    double load[kQueues] = {};
    for (size_t k = 0; k < jobs.size(); ++k) {
        int q = 0;
        if (k > 0) {
            q = 1;
            for (int t = 2; t < kQueues; ++t)
                if (load[t] < load[q]) q = t;
        }
        qof[k] = q;
        load[q] += jobs[k].cost;
    }
    hipEvent_t fork = ctx->qevents[0];
    HIPCHK(hipEventRecord(fork, os));
    bool used[kQueues] = {};
    for (size_t k = 0; k < jobs.size(); ++k) used[qof[k]] = true;
    if (used[0]) HIPCHK(hipStreamWaitEvent(ctx->qstreams[0], fork, 0));
    hipEvent_t head = ctx->qevents[1 + 2 * (size_t)n_levels + kQueues];
    std::vector<int> fine_q(n_levels, 0), coarse_q(n_levels, 0);
    for (size_t k = 0; k < jobs.size(); ++k) {
        if (k == 1)
            for (int q = 1; q < kQueues; ++q)
                if (used[q]) HIPCHK(hipStreamWaitEvent(ctx->qstreams[q], head, 0));
        const job &J = jobs[k];
        const int i = J.li;
        hipStream_t sq = ctx->qstreams[qof[k]];
        void *w = (char *)ws_dev + off[i];
        const level_layout &L = LL[i];
        const mlmc_level_opts &o = opts[i];
        const grid_layout &G = J.coarse ? L.coarse : L.fine;
        void *wg = at<void>(w, J.coarse ? L.off_coarse : L.off_fine);
        int rc = solve_grid(ctx, G, levels[i] - J.coarse, xi_dev[i], o, J.coarse ? o.eps_coarse : o.eps_fine, wg,
                            at<double>(w, J.coarse ? L.off_qc : L.off_qf), at<int32_t>(wg, G.off_iters), sq,
                            k == 0 ? head : nullptr);
        if (rc) return rc;
        if (J.coarse) {
            coarse_q[i] = qof[k];
            HIPCHK(hipEventRecord(ctx->qevents[1 + 2 * i], sq));
        } else {
            fine_q[i] = qof[k];
        }
    }
    for (int i = 0; i < n_levels; ++i) {
        if (n[i] == 0) continue;
        hipStream_t sq = ctx->qstreams[fine_q[i]];
        void *w = (char *)ws_dev + off[i];
        const level_layout &L = LL[i];
        void *wf = at<void>(w, L.off_fine);
        const uint32_t *stc = nullptr;
        const int32_t *itc = nullptr;
        if (levels[i] > 0) {
            if (coarse_q[i] != fine_q[i]) HIPCHK(hipStreamWaitEvent(sq, ctx->qevents[1 + 2 * i], 0));
            void *wc = at<void>(w, L.off_coarse);
            stc = at<uint32_t>(wc, L.coarse.off_state);
            itc = at<int32_t>(wc, L.coarse.off_iters);
        }
        HIPCHK(launch_pair_sums((int)n[i], at<double>(w, L.off_qf), levels[i] > 0 ? at<double>(w, L.off_qc) : nullptr,
                                at<uint32_t>(wf, L.fine.off_state), stc, at<int32_t>(wf, L.fine.off_iters), itc,
                                y_dev ? y_dev[i] : nullptr, nullptr, at<double>(w, L.off_sums), sq));
    }
    for (int q = 0; q < kQueues; ++q) {
        if (!used[q]) continue;
        hipEvent_t e = ctx->qevents[1 + 2 * (size_t)n_levels + q];
        HIPCHK(hipEventRecord(e, ctx->qstreams[q]));
        HIPCHK(hipStreamWaitEvent(os, e, 0));
    }
    return MLMC_OK;
}

void fill_stats(mlmc_level_stats *out, int64_t n, const double *h, double ms)
{
    memset(out, 0, sizeof *out);
    out->n = n;
    if (n > 0) {
        out->sum_y = h[0];
        out->sum_y2 = h[1];
        out->sum_qf = h[2];
        out->sum_qc = h[3];
        out->n_promoted = (int64_t)h[4];
        out->n_noconv = (int64_t)h[5];
        out->mean_iters = h[6] / (double)n;
        out->mean_iters_coarse = h[7] / (double)n;
    }
    out->gpu_ms = ms;
}

// One MLMC level on the workspace ws_dev (a caller buffer, or the library's
// scratch array for the no-allocation entry point).
int sample_level_impl(mlmc_ctx *ctx, int32_t level, int64_t n, const double *xi_dev,
                      const mlmc_level_opts *opts, void *ws_dev, size_t ws_bytes,
                      double *q_fine_dev, double *q_coarse_dev, double *y_dev,
                      uint8_t *status_dev, mlmc_level_stats *stats_host, void *stream)
{
    int rc = check_level(ctx, level);
    if (rc) return rc;
    if ((rc = check_opts(ctx, opts, level, true))) return rc;
    if (n < 0 || n > 4000000) return fail(ctx, MLMC_EINVAL, "bad sample count (0..4e6)");
    if (n > 0 && (!xi_dev || !ws_dev)) return fail(ctx, MLMC_EINVAL, "null pointer");
    if (((uintptr_t)ws_dev & 255) != 0) return fail(ctx, MLMC_EINVAL, "workspace not 256-byte aligned");
    if (!aligned(xi_dev, 8) || !aligned(q_fine_dev, 8) || !aligned(q_coarse_dev, 8) || !aligned(y_dev, 8))
        return fail(ctx, MLMC_EINVAL, "sample_level: misaligned pointer");
    const level_layout LL = make_level_layout(ctx->cfg, level, n, *opts);
    if (ws_bytes < LL.bytes) return fail(ctx, MLMC_ENOMEM, "workspace %zu < %zu bytes", ws_bytes, LL.bytes);
    hipStream_t st = (hipStream_t)stream;
    if (stats_host) HIPCHK(hipEventRecord(ctx->ev0, st));
    rc = level_enqueue(ctx, level, n, xi_dev, *opts, ws_dev, LL, q_fine_dev, q_coarse_dev, y_dev, status_dev,
                       st, st, nullptr);
    if (rc) return rc;
    if (stats_host) {
        HIPCHK(hipEventRecord(ctx->ev1, st));
        if (n > 0) HIPCHK(hipMemcpyAsync(ctx->h_sums, at<double>(ws_dev, LL.off_sums), 8 * 8, hipMemcpyDeviceToHost, st));
        HIPCHK(hipStreamSynchronize(st));
        float ms = 0.f;
        HIPCHK(hipEventElapsedTime(&ms, ctx->ev0, ctx->ev1));
        fill_stats(stats_host, n, ctx->h_sums, ms);
        return stats_host->n_noconv > 0 ? MLMC_ENOCONV : MLMC_OK;
    }
    return MLMC_OK;
}

}  // namespace

// ================================================================ C ABI

extern "C" {

int mlmc_create(const mlmc_config *cfg, mlmc_ctx **out)
{
    if (!cfg || !out) return MLMC_EINVAL;
    *out = nullptr;
    const mlmc_config &c = *cfg;
    if (c.m != 2 || !is_pow2(c.n0) || c.n0 < 4 || c.L_max < 0 || (c.n0 << c.L_max) > 256 ||
        c.K < 1 || c.K > 512 || !(c.sigma2 >= 0.0) || c.field < 0 || c.field > 1 || c.disc < 0 || c.disc > 1 ||
        (c.field == 0 && !(c.corr_len > 0.0)) || (c.field == 1 && !(c.field_q >= 0.0 && c.field_q < 1e3)) ||
        !std::isfinite(c.f) ||
        !(c.k_p > 0.0 && c.k_p < 1.0) || c.ir_max_iter < 0 || c.L_max > 15 || !(c.alpha > 0.0) ||
        !(c.beta > 0.0) || !(c.gamma > 0.0) || !std::isfinite(c.alpha + c.beta + c.gamma))
        return MLMC_EINVAL;
    mlmc_ctx *ctx = new mlmc_ctx();
    ctx->cfg = c;
    if (hipGetDevice(&ctx->device) != hipSuccess ||
        scratch_device_ptr(ctx->device, &ctx->scratch) != hipSuccess) {
        delete ctx;
        return MLMC_EHIP;
    }
    std::vector<std::vector<double>> ph;
    int rc = build_phit(ctx, ph);
    if (rc) {
        delete ctx;
        return rc;
    }
    ctx->phit.assign(c.L_max + 1, nullptr);
    for (int l = 0; l <= c.L_max; ++l) {
        if (hipMalloc(&ctx->phit[l], ph[l].size() * 8) != hipSuccess ||
            hipMemcpy(ctx->phit[l], ph[l].data(), ph[l].size() * 8, hipMemcpyHostToDevice) != hipSuccess) {
            mlmc_destroy(ctx);
            return MLMC_EHIP;
        }
    }
    if (hipMalloc(&ctx->d_counter, 64) != hipSuccess || hipMalloc(&ctx->d_sums, 16 * 8) != hipSuccess ||
        hipHostMalloc(&ctx->h_counter, 64, 0) != hipSuccess ||
        hipHostMalloc(&ctx->h_sums, 16 * 8, 0) != hipSuccess || hipEventCreate(&ctx->ev0) != hipSuccess ||
        hipEventCreate(&ctx->ev1) != hipSuccess) {
        mlmc_destroy(ctx);
        return MLMC_EHIP;
    }
    *out = ctx;
    return MLMC_OK;
}

int mlmc_destroy(mlmc_ctx *ctx)
{
    if (!ctx) return MLMC_EINVAL;
    for (double *p : ctx->phit)
        if (p) (void)hipFree(p);
    if (ctx->d_counter) (void)hipFree(ctx->d_counter);
    if (ctx->d_sums) (void)hipFree(ctx->d_sums);
    if (ctx->h_counter) (void)hipHostFree(ctx->h_counter);
    if (ctx->h_sums) (void)hipHostFree(ctx->h_sums);
    for (auto &r : ctx->prof) {
        (void)hipEventDestroy(r.a);
        (void)hipEventDestroy(r.b);
    }
    for (hipEvent_t e : ctx->ev_pool) (void)hipEventDestroy(e);
    for (hipEvent_t e : ctx->levents) (void)hipEventDestroy(e);
    for (hipStream_t s2 : ctx->lstreams) (void)hipStreamDestroy(s2);
    for (hipEvent_t e : ctx->qevents) (void)hipEventDestroy(e);
    if (ctx->est_buf) (void)hipFree(ctx->est_buf);
    for (hipStream_t s2 : ctx->qstreams) (void)hipStreamDestroy(s2);
    if (ctx->cap_stream) (void)hipStreamDestroy(ctx->cap_stream);
    if (ctx->graph_exec) (void)hipGraphExecDestroy(ctx->graph_exec);
    if (ctx->graph) (void)hipGraphDestroy(ctx->graph);
    if (ctx->ev0) (void)hipEventDestroy(ctx->ev0);
    if (ctx->ev1) (void)hipEventDestroy(ctx->ev1);
    delete ctx;
    return MLMC_OK;
}

const char *mlmc_last_error(const mlmc_ctx *ctx) { return ctx ? ctx->err.c_str() : "null context"; }

int32_t mlmc_level_cells(const mlmc_ctx *ctx, int32_t level)
{
    if (!ctx || level < 0 || level > ctx->cfg.L_max) return -1;
    return ctx->cfg.n0 << level;
}

int mlmc_accuracy_targets(const mlmc_ctx *ctx, int32_t L, double *eps_out)
{
    if (!ctx || !eps_out || L < 0 || L > 15) return MLMC_EINVAL;
    // Sec. 4.3's precision choice with the error lemma's exponents of delta
    // (1 in the bias, 2 in the variance): (k_p h^beta)^(1/2) below the finest
    // level, the smaller of that and k_p h^alpha on it.
    const mlmc_config &c = ctx->cfg;
    for (int l = 0; l <= L; ++l) {
        const double h = 1.0 / ((double)c.n0 * std::pow(2.0, l));
        const double ev = std::sqrt(c.k_p * std::pow(h, c.beta));
        eps_out[l] = l < L ? ev : std::min(ev, c.k_p * std::pow(h, c.alpha));
    }
    return MLMC_OK;
}

int mlmc_get_kl_basis(const mlmc_ctx *cctx, int32_t level, double *phit_dev, void *stream)
{
    mlmc_ctx *ctx = const_cast<mlmc_ctx *>(cctx);
    if (!ctx || level < 0 || level > ctx->cfg.L_max || !phit_dev)
        return fail(ctx, MLMC_EINVAL, "get_kl_basis: bad arguments");
    const int n = ctx->cfg.n0 << level;
    const size_t bytes = (size_t)ctx->cfg.K * (n + 1) * (n + 1) * 8;
    HIPCHK(hipMemcpyAsync(phit_dev, ctx->phit[level], bytes, hipMemcpyDeviceToDevice, (hipStream_t)stream));
    return MLMC_OK;
}

size_t mlmc_workspace_bytes(const mlmc_ctx *ctx, int32_t level, int64_t n_samples,
                            const mlmc_level_opts *opts)
{
    if (!ctx || !opts || level < 0 || level > ctx->cfg.L_max || n_samples < 0) return 0;
    return make_level_layout(ctx->cfg, level, n_samples, *opts).bytes;
}

int mlmc_set_seed(mlmc_ctx *ctx, uint64_t seed)
{
    if (!ctx) return MLMC_EINVAL;
    ctx->cfg.seed = seed;
    return MLMC_OK;
}

int mlmc_fill_xi(const mlmc_ctx *cctx, int32_t level, int64_t first_sample, int64_t n,
                 double *xi_dev, void *stream)
{
    mlmc_ctx *ctx = const_cast<mlmc_ctx *>(cctx);
    if (!ctx || level < 0 || level > 32767 || first_sample < 0 || n < 0 ||
        first_sample + n > (int64_t)1 << 32 || (!xi_dev && n > 0) || !aligned(xi_dev, 8))
        return fail(ctx, MLMC_EINVAL, "fill_xi: bad arguments");
    HIPCHK(launch_fill_xi(ctx->cfg.seed, level, first_sample, n, ctx->cfg.K, xi_dev, (hipStream_t)stream));
    return MLMC_OK;
}

int mlmc_solve(mlmc_ctx *ctx, int32_t level, int64_t n, const double *xi_dev,
               const mlmc_level_opts *opts, void *ws_dev, size_t ws_bytes, double *q_dev,
               double *u_dev, uint8_t *status_dev, int32_t *iters_dev, void *stream)
{
    int rc = check_level(ctx, level);
    if (rc) return rc;
    if ((rc = check_opts(ctx, opts, level, false))) return rc;
    if (n < 0 || n > 4000000) return fail(ctx, MLMC_EINVAL, "bad sample count (0..4e6)");
    if (n == 0) return MLMC_OK;
    if (!xi_dev || !ws_dev || !q_dev) return fail(ctx, MLMC_EINVAL, "null pointer");
    if (((uintptr_t)ws_dev & 255) != 0) return fail(ctx, MLMC_EINVAL, "workspace not 256-byte aligned");
    if (!aligned(xi_dev, 8) || !aligned(q_dev, 8) || !aligned(u_dev, 8) || !aligned(iters_dev, 4))
        return fail(ctx, MLMC_EINVAL, "solve: misaligned pointer");
    const level_layout LL = make_level_layout(ctx->cfg, level, n, *opts);
    if (ws_bytes < LL.bytes) return fail(ctx, MLMC_ENOMEM, "workspace %zu < %zu bytes", ws_bytes, LL.bytes);
    hipStream_t st = (hipStream_t)stream;
    const grid_layout &L = LL.fine;
    void *ws = at<void>(ws_dev, LL.off_fine);
    int32_t *it = at<int32_t>(ws, L.off_iters);
    rc = solve_grid(ctx, L, level, xi_dev, *opts, opts->eps_fine, ws, q_dev, it, st);
    if (rc) return rc;
    if (u_dev) HIPCHK(launch_unpad(L.n, (int)n, at<double>(ws, L.off_x), u_dev, st));
    if (iters_dev) HIPCHK(hipMemcpyAsync(iters_dev, it, n * 4, hipMemcpyDeviceToDevice, st));
    double *sums = at<double>(ws_dev, LL.off_sums);
    HIPCHK(launch_pair_sums((int)n, q_dev, nullptr, at<uint32_t>(ws, L.off_state), nullptr, it, nullptr,
                            nullptr, status_dev, sums, st));
    HIPCHK(hipMemcpyAsync(ctx->h_sums, sums, 8 * 8, hipMemcpyDeviceToHost, st));
    HIPCHK(hipStreamSynchronize(st));
    return ctx->h_sums[5] > 0 ? MLMC_ENOCONV : MLMC_OK;
}

int mlmc_sample_level(mlmc_ctx *ctx, int32_t level, int64_t n, const double *xi_dev,
                      const mlmc_level_opts *opts, void *ws_dev, size_t ws_bytes,
                      double *q_fine_dev, double *q_coarse_dev, double *y_dev,
                      uint8_t *status_dev, mlmc_level_stats *stats_host, void *stream)
{
    return sample_level_impl(ctx, level, n, xi_dev, opts, ws_dev, ws_bytes, q_fine_dev, q_coarse_dev, y_dev,
                             status_dev, stats_host, stream);
}

int mlmc_sample_level_noalloc(mlmc_ctx *ctx, int32_t level, int64_t n, const double *xi_dev,
                              const mlmc_level_opts *opts, double *q_fine_dev, double *q_coarse_dev,
                              double *y_dev, uint8_t *status_dev, mlmc_level_stats *stats_host,
                              void *stream)
{
    int rc = check_level(ctx, level);
    if (rc) return rc;
    if ((rc = check_opts(ctx, opts, level, true))) return rc;
    if (n < 0 || n > 4000000) return fail(ctx, MLMC_EINVAL, "bad sample count (0..4e6)");
    if (!ctx->scratch) return fail(ctx, MLMC_EHIP, "no scratch address for device %d", ctx->device);
    const size_t need = make_level_layout(ctx->cfg, level, n, *opts).bytes;
    if (need > kNoallocScratchBytes)
        return fail(ctx, MLMC_ENOMEM, "sample_level_noalloc: %lld samples on level %d need %zu bytes, the scratch holds %zu",
                    (long long)n, level, need, kNoallocScratchBytes);
    // the event-timed kernel records create events on demand: off for this call
    const bool prof = ctx->prof_on;
    ctx->prof_on = false;
    rc = sample_level_impl(ctx, level, n, xi_dev, opts, ctx->scratch, kNoallocScratchBytes, q_fine_dev,
                           q_coarse_dev, y_dev, status_dev, stats_host, stream);
    ctx->prof_on = prof;
    return rc;
}

size_t mlmc_levels_workspace_bytes(const mlmc_ctx *ctx, int32_t n_levels, const int32_t *levels,
                                   const int64_t *n, const mlmc_level_opts *opts)
{
    if (!ctx || n_levels < 1 || n_levels > 16 || !levels || !n || !opts) return 0;
    size_t tot = 0;
    for (int i = 0; i < n_levels; ++i) {
        if (levels[i] < 0 || levels[i] > ctx->cfg.L_max || n[i] < 0) return 0;
        tot += align256(make_level_layout(ctx->cfg, levels[i], n[i], opts[i]).bytes);
    }
    return tot;
}

int mlmc_sample_levels(mlmc_ctx *ctx, int32_t n_levels, const int32_t *levels, const int64_t *n,
                       const double *const *xi_dev, const mlmc_level_opts *opts, void *ws_dev,
                       size_t ws_bytes, double *const *y_dev, mlmc_level_stats *stats_host,
                       int32_t use_graph, void *stream)
{
    if (!ctx) return MLMC_EINVAL;
    if (n_levels < 1 || n_levels > 16 || !levels || !n || !xi_dev || !opts || !ws_dev)
        return fail(ctx, MLMC_EINVAL, "sample_levels: bad arguments");
    if (((uintptr_t)ws_dev & 255) != 0) return fail(ctx, MLMC_EINVAL, "workspace not 256-byte aligned");
    std::vector<level_layout> LL(n_levels);
    std::vector<size_t> off(n_levels);
    size_t tot = 0;
    for (int i = 0; i < n_levels; ++i) {
        int rc = check_level(ctx, levels[i]);
        if (rc) return rc;
        if ((rc = check_opts(ctx, &opts[i], levels[i], true))) return rc;
        if (n[i] < 0 || n[i] > 4000000) return fail(ctx, MLMC_EINVAL, "bad sample count (0..4e6)");
        if (n[i] > 0 && !xi_dev[i]) return fail(ctx, MLMC_EINVAL, "null xi");
        if (!aligned(xi_dev[i], 8) || (y_dev && !aligned(y_dev[i], 8)))
            return fail(ctx, MLMC_EINVAL, "sample_levels: misaligned pointer");
        LL[i] = make_level_layout(ctx->cfg, levels[i], n[i], opts[i]);
        off[i] = tot;
        tot += align256(LL[i].bytes);
    }
    if (ws_bytes < tot) return fail(ctx, MLMC_ENOMEM, "workspace %zu < %zu bytes", ws_bytes, tot);
    hipStream_t st = (hipStream_t)stream;
    // streams and events for the fork/join (created once, default priority)
    const size_t need = 2 * (size_t)n_levels;
    while (ctx->lstreams.size() < need) {
        hipStream_t s2;
        HIPCHK(hipStreamCreateWithFlags(&s2, hipStreamNonBlocking));
        ctx->lstreams.push_back(s2);
    }
    while (ctx->levents.size() < 2 * need + 1) {
        hipEvent_t e;
        HIPCHK(hipEventCreateWithFlags(&e, hipEventDisableTiming));
        ctx->levents.push_back(e);
    }
    // os: the stream the fork starts from and the join ends on
    auto enqueue_all = [&](hipStream_t os) -> int {
        hipEvent_t fork = ctx->levents[0];
        HIPCHK(hipEventRecord(fork, os));
        for (int i = 0; i < n_levels; ++i) {
            hipStream_t sf = ctx->lstreams[2 * i], scs = ctx->lstreams[2 * i + 1];
            HIPCHK(hipStreamWaitEvent(sf, fork, 0));
            // the coarse stream joins only when it has work (every fork is joined back)
            if (levels[i] > 0 && n[i] > 0) HIPCHK(hipStreamWaitEvent(scs, fork, 0));
            void *w = (char *)ws_dev + off[i];
            int rc = level_enqueue(ctx, levels[i], n[i], xi_dev[i], opts[i], w, LL[i], nullptr, nullptr,
                                   y_dev ? y_dev[i] : nullptr, nullptr, sf, scs, ctx->levents[1 + 2 * i]);
            if (rc) return rc;
            HIPCHK(hipEventRecord(ctx->levents[2 + 2 * i], sf));
            HIPCHK(hipStreamWaitEvent(os, ctx->levents[2 + 2 * i], 0));

        }
        return MLMC_OK;
    };
    if (stats_host) HIPCHK(hipEventRecord(ctx->ev0, st));
    if (use_graph) {
        std::vector<uintptr_t> key = {(uintptr_t)n_levels, (uintptr_t)ws_dev};
        for (int i = 0; i < n_levels; ++i) {
            key.push_back((uintptr_t)levels[i]);
            key.push_back((uintptr_t)n[i]);
            key.push_back((uintptr_t)xi_dev[i]);
            key.push_back(y_dev ? (uintptr_t)y_dev[i] : 0);
            const unsigned char *ob = (const unsigned char *)&opts[i];
            for (size_t b = 0; b < sizeof(mlmc_level_opts); b += sizeof(uintptr_t)) {
                uintptr_t v = 0;
                memcpy(&v, ob + b, std::min(sizeof(uintptr_t), sizeof(mlmc_level_opts) - b));
                key.push_back(v);
            }
        }
        for (auto &row : ctx->ir_variant)
            for (int v : row) key.push_back((uintptr_t)v);
        if (!ctx->graph_exec || key != ctx->graph_key) {
            if (ctx->graph_exec) (void)hipGraphExecDestroy(ctx->graph_exec);
            if (ctx->graph) (void)hipGraphDestroy(ctx->graph);
            ctx->graph_exec = nullptr;
            ctx->graph = nullptr;
            // captured on a stream of the context (the caller's stream may be
            // the legacy null stream, which cannot be captured); the graph is
            // then launched on the caller's stream
            if (!ctx->cap_stream) HIPCHK(hipStreamCreateWithFlags(&ctx->cap_stream, hipStreamNonBlocking));
            ctx->capturing = true;
            HIPCHK(hipStreamBeginCapture(ctx->cap_stream, hipStreamCaptureModeThreadLocal));
            int rc = enqueue_all(ctx->cap_stream);
            hipGraph_t gr = nullptr;
            const hipError_t ec = hipStreamEndCapture(ctx->cap_stream, &gr);
            ctx->capturing = false;
            if (rc) {
                if (gr) (void)hipGraphDestroy(gr);
                return rc;
            }
            if (ec != hipSuccess) return fail(ctx, MLMC_EHIP, "graph capture: %s", hipGetErrorString(ec));
            ctx->graph = gr;
            HIPCHK(hipGraphInstantiate(&ctx->graph_exec, gr, nullptr, nullptr, 0));
            ctx->graph_key = key;
        }
        HIPCHK(hipGraphLaunch(ctx->graph_exec, st));
    } else {
        int rc = enqueue_levels_queued(ctx, n_levels, levels, n, xi_dev, opts, ws_dev, LL, off, y_dev, st);
        if (rc) return rc;
    }
    if (stats_host) {
        HIPCHK(hipEventRecord(ctx->ev1, st));
        HIPCHK(hipStreamSynchronize(st));
        float ms = 0.f;
        HIPCHK(hipEventElapsedTime(&ms, ctx->ev0, ctx->ev1));
        int any_noconv = 0;
        for (int i = 0; i < n_levels; ++i) {
            double h[8] = {};
            if (n[i] > 0)
                HIPCHK(hipMemcpy(h, at<double>((char *)ws_dev + off[i], LL[i].off_sums), 8 * 8, hipMemcpyDeviceToHost));
            fill_stats(&stats_host[i], n[i], h, ms);
            any_noconv |= stats_host[i].n_noconv > 0;
        }
        return any_noconv ? MLMC_ENOCONV : MLMC_OK;
    }
    return MLMC_OK;
}

int mlmc_autotune(mlmc_ctx *ctx, int32_t level, int64_t n, const double *xi_dev,
                  const mlmc_level_opts *opts, void *ws_dev, size_t ws_bytes, int32_t *chosen,
                  void *stream)
{
    int rc = check_level(ctx, level);
    if (rc) return rc;
    if ((rc = check_opts(ctx, opts, level, true))) return rc;
    if (n < 1 || !xi_dev || !ws_dev) return fail(ctx, MLMC_EINVAL, "autotune: bad arguments");
    const level_layout LL = make_level_layout(ctx->cfg, level, n, *opts);
    if (ws_bytes < LL.bytes) return fail(ctx, MLMC_ENOMEM, "workspace %zu < %zu bytes", ws_bytes, LL.bytes);
    if (is_iterative(opts->solver)) return MLMC_OK;
    hipStream_t st = (hipStream_t)stream;
    const int dt = opts->solver == MLMC_DIRECT ? MLMC_F64 : opts->factor_dtype;
    const bool was = ctx->prof_on;
    ctx->prof_on = false;
    for (int g = 0; g < (level > 0 ? 2 : 1); ++g) {
        const int lv = level - g, nn = ctx->cfg.n0 << lv;
        const grid_layout &L = g ? LL.coarse : LL.fine;
        void *w = at<void>(ws_dev, g ? LL.off_coarse : LL.off_fine);
        // candidates: the refinement kernel's waves per row pair (grids from
        // n = 64) and, for the FP16/BF16 factors on the MFMA grids (n >= 32),
        // products in the storage format or in FP32; each timed as the whole
        // solve of the grid (factor and refinement: a faster factorisation
        // may cost corrections)
        const int nir = (use_blk(dt, nn) && nn >= 64) ? 2 : 0;
        const int nfv = ((dt == MLMC_F16 || dt == MLMC_BF16) && nn >= 32) ? 2 : 1;
        int best = 0;
        if (nir > 0 || nfv > 1) {
            float best_ms = 1e30f;
            int best_ir = 0, best_fv = 0;
            for (int fv = 0; fv < nfv; ++fv)
                for (int var = (nir ? 1 : 0); var <= nir; ++var) {
                    ctx->ir_variant[dt][ilog2(nn)] = var;
                    ctx->factor_variant[dt][ilog2(nn)] = fv;
                    for (int rep = 0; rep < 3; ++rep) {
                        if (rep == 1) HIPCHK(hipEventRecord(ctx->ev0, st));
                        rc = solve_grid(ctx, L, lv, xi_dev, *opts, g ? opts->eps_coarse : opts->eps_fine, w,
                                        at<double>(ws_dev, g ? LL.off_qc : LL.off_qf), nullptr, st);
                        if (rc) return rc;
                    }
                    HIPCHK(hipEventRecord(ctx->ev1, st));
                    HIPCHK(hipEventSynchronize(ctx->ev1));
                    float ms = 0.f;
                    HIPCHK(hipEventElapsedTime(&ms, ctx->ev0, ctx->ev1));
                    if (ms < best_ms) {
                        best_ms = ms;
                        best_ir = var;
                        best_fv = fv;
                    }
                }
            ctx->ir_variant[dt][ilog2(nn)] = best_ir;
            ctx->factor_variant[dt][ilog2(nn)] = best_fv;
            best = best_ir | (best_fv << 4);
        }
        if (chosen) chosen[g] = best;
    }
    ctx->prof_on = was;
    return MLMC_OK;
}

int mlmc_estimate(mlmc_ctx *ctx, double tol, int32_t n_init, const mlmc_dtype *dtype_per_level,
                  mlmc_solver solver, int32_t mixed, mlmc_result *out, void *stream)
{
    return mlmc_estimate_resumable(ctx, tol, n_init, dtype_per_level, solver, mixed, nullptr, 0, nullptr, out,
                                   stream);
}

int mlmc_estimate_resumable(mlmc_ctx *ctx, double tol, int32_t n_init, const mlmc_dtype *dtype_per_level,
                            mlmc_solver solver, int32_t mixed, const mlmc_estimate_state *resume,
                            int32_t max_rounds, mlmc_estimate_state *state_out, mlmc_result *out,
                            void *stream)
{
    if (!ctx || !out || !(tol > 0.0) || n_init < 2 || ctx->cfg.L_max < 1 || ctx->cfg.L_max > 15)
        return fail(ctx, MLMC_EINVAL, "estimate: bad arguments");
    if (!dtype_per_level && solver == MLMC_DIRECT_IR)
        return fail(ctx, MLMC_EINVAL, "estimate: dtype_per_level is NULL");
    const auto t0 = std::chrono::steady_clock::now();
    hipStream_t st = (hipStream_t)stream;
    const mlmc_config &c = ctx->cfg;
    // tolerance of every solve of standard MLMC with an iterative solver
    const double std_eps = (!mixed && is_iterative(solver)) ? (c.std_eps > 0.0 ? c.std_eps : 1e-6) : 0.0;
    const int Lmax = c.L_max;
    // Per-level chunk: as many samples as fit a per-level workspace budget, so
    // that the fine levels fill the GPU.  Each level has its own workspace and
    // xi buffer and, within a round, streams its chunks back to back on one
    // of the context's queue streams, so that a level with many chunks (the
    // coarsest) and one with a few long ones (the finest) run side by side
    // rather than in lockstep; every chunk's level sums are copied to pinned
    // host memory and added in chunk order after the round's one
    // synchronisation.
    // A level's budget may grow to big_budget when that lets the chunk hold
    // the initial N_l (rounded up to a power of two), so that a newly added
    // fine level (few samples, each a long latency-bound chain) is one launch
    // rather than several in sequence.
    const int64_t chunk_max = 1 << 18;
    const size_t level_budget = (size_t)8 << 30, big_budget = (size_t)32 << 30;
    int64_t min_chunk = 1;
    while (min_chunk < n_init) min_chunk *= 2;
    std::vector<int64_t> chunk(Lmax + 1);
    std::vector<mlmc_level_opts> lopt(Lmax + 1);
    size_t ws_bytes = 0, xi_bytes = 0;
    std::vector<size_t> xi_off(Lmax + 1), ws_off(Lmax + 1);
    for (int l = 0; l <= Lmax; ++l) {
        mlmc_level_opts o{};
        o.factor_dtype = dtype_per_level ? dtype_per_level[l] : MLMC_F64;
        // standard MLMC: FP64 direct solves, or the iterative solver at the
        // fixed tolerance std_eps (the paper's standard MLMC with MINRES)
        o.solver = mixed ? solver : (is_iterative(solver) ? solver : MLMC_DIRECT);
        o.promote = 1;
        if (int rc_o = check_opts(ctx, &o, l, true)) return rc_o;
        int64_t ch = chunk_max;
        while (ch > 16) {
            const size_t b = make_level_layout(c, l, ch, o).bytes;
            if (b <= level_budget || (ch <= min_chunk && b <= big_budget)) break;
            ch /= 2;
        }
        chunk[l] = ch;
        lopt[l] = o;
        ws_off[l] = ws_bytes;
        ws_bytes += align256(make_level_layout(c, l, ch, o).bytes);
        xi_off[l] = xi_bytes;
        xi_bytes += align256((size_t)ch * c.K * 8);
    }
    const size_t need = align256(ws_bytes) + xi_bytes;
    if (ctx->est_bytes < need) {
        if (ctx->est_buf) (void)hipFree(ctx->est_buf);
        ctx->est_buf = nullptr;
        ctx->est_bytes = 0;
        if (hipMalloc(&ctx->est_buf, need) != hipSuccess)
            return fail(ctx, MLMC_ENOMEM, "estimate: out of device memory (%zu bytes)", need);
        ctx->est_bytes = need;
    }
    void *ws = ctx->est_buf;
    char *xi = (char *)ctx->est_buf + align256(ws_bytes);
    auto cost = [&](int l) {
        auto f = [&](int n) { return std::pow((double)(n - 1), c.gamma); };
        return f(c.n0 << l) + (l > 0 ? f(c.n0 << (l - 1)) : 0.0);
    };
    int L = 1;
    std::vector<int64_t> N = {n_init, n_init}, done = {0, 0};
    std::vector<double> s1 = {0, 0}, s2 = {0, 0};
    std::vector<double> yhat, var;
    int32_t dts[16] = {};
    for (int l = 0; l <= Lmax; ++l) dts[l] = dtype_per_level ? (int32_t)dtype_per_level[l] : 0;
    int start_round = 0;
    if (resume) {
        const mlmc_estimate_state &R = *resume;
        bool ok = R.L >= 1 && R.L <= Lmax && R.rounds >= 0 && R.tol == tol && R.n_init == n_init &&
                  R.mixed == mixed && R.solver == (int32_t)solver && R.seed == c.seed;
        for (int l = 0; l <= Lmax && ok; ++l) ok = R.dtype[l] == dts[l];
        for (int l = 0; l <= R.L && ok; ++l)
            ok = R.done[l] >= 0 && R.N[l] >= 0 && std::isfinite(R.s1[l]) && std::isfinite(R.s2[l]);
        if (!ok) return fail(ctx, MLMC_EINVAL, "estimate: the resume state does not match this call or context");
        L = R.L;
        N.assign(R.N, R.N + L + 1);
        done.assign(R.done, R.done + L + 1);
        s1.assign(R.s1, R.s1 + L + 1);
        s2.assign(R.s2, R.s2 + L + 1);
        start_round = R.rounds;
    }
    const double bias_c = (std::pow((double)c.m, c.alpha) - 1.0) / std::sqrt(2.0) * tol;
    double gpu_ms = resume ? resume->gpu_ms : 0.0;
    double *hbuf = nullptr;  // pinned: 8 sums per chunk of a round
    int hcap = 0;
    int rc = MLMC_OK;
    int converged = 0;
    // per level: samples re-solved in FP64 and samples that missed their
    // target; the latter, or non-finite level sums, end the call (every Y_l
    // of Algorithm 4.1 must reach its accuracy)
    int64_t n_prom[16] = {}, n_nc[16] = {};
    if (resume)
        for (int l = 0; l <= Lmax; ++l) {
            n_prom[l] = resume->n_promoted[l];
            n_nc[l] = resume->n_noconv[l];
        }
    bool inexact = false, paused = false;
    int rounds = start_round;
    for (int round = start_round; round < 200; ++round) {
        double eps[16];
        mlmc_accuracy_targets(ctx, L, eps);
        // Algorithm 4.1 adds level L + 1 (with n_init samples) when |Y_L| is
        // above the bias bound after a round.  That decision is known as soon as
        // level L's samples of the round are in (at once if it has none to add):
        // the new level's first samples then run in this round, beside the other
        // levels' top-ups, with the accuracy targets of L + 1 levels.  The
        // decisions and sums are those of running them in the next round.
        auto next_level_due = [&](double s1L, int64_t doneL) {
            return L < Lmax && doneL > 0 && std::fabs(s1L / (double)doneL) > bias_c;
        };
        double eps_next[16] = {};
        if (L < Lmax) mlmc_accuracy_targets(ctx, L + 1, eps_next);
        struct job { int l; int64_t from, to; double ef, ec; };
        const job next_job{L + 1, 0, n_init, mixed ? eps_next[L + 1] : std_eps, mixed ? eps_next[L] : std_eps};
        const bool early = N[L] <= done[L] && next_level_due(s1[L], done[L]);
        std::vector<job> jobs;
        // finest first: issuing level 0's many chunks takes the host milliseconds
        if (early) jobs.push_back(next_job);
        for (int l = L; l >= 0; --l)
            if (N[l] > done[l])
                jobs.push_back({l, done[l], N[l], mixed ? eps[l] : std_eps,
                                mixed ? (l > 0 ? eps[l - 1] : 0.0) : (l > 0 ? std_eps : 0.0)});
        auto job_chunks = [&](const job &jb) { return (int)((jb.to - jb.from + chunk[jb.l] - 1) / chunk[jb.l]); };
        // top every level up to N_l
        auto round_enqueue = [&](std::vector<std::pair<int, int64_t>> &recs) -> int {
            int nchunks = 0;
            for (const job &jb : jobs) nchunks += job_chunks(jb);
            if (nchunks == 0) return MLMC_OK;
            if (!early && L < Lmax) nchunks += job_chunks(next_job);
            if (int e = ensure_queues(ctx, 2 + kQueues)) return e;
            if (nchunks > hcap) {
                if (hbuf) (void)hipHostFree(hbuf);
                hbuf = nullptr;
                hcap = 0;
                HIPCHK(hipHostMalloc((void **)&hbuf, (size_t)nchunks * 8 * sizeof(double), 0));
                hcap = nchunks;
            }
            hipEvent_t fork = ctx->qevents[0];
            HIPCHK(hipEventRecord(ctx->ev0, st));
            HIPCHK(hipEventRecord(fork, st));
            bool used[kQueues] = {};
            // The first three context streams have hardware queues of their own
            // (the fourth shares one): level 0 (the most chunks) and the finest
            // level with work (the longest per-sample chain) take one each, the
            // levels between share the rest.
            const int top = jobs.front().l;
            auto level_queue = [&](int l) { return l == 0 ? 0 : (l >= top ? 1 : 2 + (l & 1)); };
            // Level L's decision is taken as soon as its samples are in: the host
            // polls its stream between the chunks it issues for the other levels
            // (and waits for it at the end of issuing).
            const bool probe = !early && L < Lmax && top == L;
            bool probed = false;
            hipEvent_t evL = ctx->qevents[1 + kQueues];
            std::function<int(const job &)> enqueue_job;
            auto poll = [&](bool block) -> int {
                if (!probe || probed) return MLMC_OK;
                if (block) {
                    HIPCHK(hipEventSynchronize(evL));
                } else {
                    const hipError_t q = hipEventQuery(evL);
                    if (q == hipErrorNotReady) return MLMC_OK;
                    HIPCHK(q);
                }
                probed = true;
                double s1L = s1[L];
                int64_t dL = done[L];
                for (size_t k = 0; k < recs.size(); ++k)
                    if (recs[k].first == L) {
                        s1L += hbuf[8 * k];
                        dL += recs[k].second;
                    }
                return next_level_due(s1L, dL) ? enqueue_job(next_job) : MLMC_OK;
            };
            enqueue_job = [&](const job &jb) -> int {
                const int l = jb.l;
                const int q = level_queue(l);
                hipStream_t sl = ctx->qstreams[q];
                if (!used[q]) HIPCHK(hipStreamWaitEvent(sl, fork, 0));
                used[q] = true;
                mlmc_level_opts o = lopt[l];
                o.eps_fine = jb.ef;
                o.eps_coarse = jb.ec;
                void *wl = (char *)ws + ws_off[l];
                double *xl = (double *)(xi + xi_off[l]);
                for (int64_t d0 = jb.from; d0 < jb.to; d0 += chunk[l]) {
                    const int64_t cnt = std::min<int64_t>(jb.to - d0, chunk[l]);
                    if (int e = mlmc_fill_xi(ctx, l, d0, cnt, xl, sl)) return e;
                    const level_layout LLc = make_level_layout(c, l, cnt, o);
                    if (int e = level_enqueue(ctx, l, cnt, xl, o, wl, LLc, nullptr, nullptr, nullptr, nullptr, sl,
                                              sl, nullptr))
                        return e;
                    HIPCHK(hipMemcpyAsync(hbuf + 8 * recs.size(), at<double>(wl, LLc.off_sums), 8 * sizeof(double),
                                          hipMemcpyDeviceToHost, sl));
                    recs.push_back({l, cnt});
                    if (l < L)
                        if (int e = poll(false)) return e;
                }
                if (probe && l == L) HIPCHK(hipEventRecord(evL, sl));
                return MLMC_OK;
            };
            for (const job &jb : jobs)
                if (int e = enqueue_job(jb)) return e;
            if (int e = poll(true)) return e;
            for (int q = 0; q < kQueues; ++q) {
                if (!used[q]) continue;
                HIPCHK(hipEventRecord(ctx->qevents[1 + q], ctx->qstreams[q]));
                HIPCHK(hipStreamWaitEvent(st, ctx->qevents[1 + q], 0));
            }
            HIPCHK(hipEventRecord(ctx->ev1, st));
            HIPCHK(hipStreamSynchronize(st));
            float ms = 0.f;
            HIPCHK(hipEventElapsedTime(&ms, ctx->ev0, ctx->ev1));
            gpu_ms += ms;
            return MLMC_OK;
        };
        std::vector<std::pair<int, int64_t>> recs;
        rc = round_enqueue(recs);
        if (rc < 0) break;
        rc = MLMC_OK;
        int64_t next_done = 0;
        double next_s1 = 0.0, next_s2 = 0.0;
        for (size_t k = 0; k < recs.size(); ++k) {
            const int l = recs[k].first;
            n_prom[l] += (int64_t)hbuf[8 * k + 4];
            n_nc[l] += (int64_t)hbuf[8 * k + 5];
            if (hbuf[8 * k + 5] != 0.0 || !std::isfinite(hbuf[8 * k]) || !std::isfinite(hbuf[8 * k + 1]))
                inexact = true;
            if (l > L) {
                next_s1 += hbuf[8 * k];
                next_s2 += hbuf[8 * k + 1];
                next_done += recs[k].second;
                continue;
            }
            s1[l] += hbuf[8 * k];
            s2[l] += hbuf[8 * k + 1];
            done[l] += recs[k].second;
        }
        yhat.assign(L + 1, 0.0);
        var.assign(L + 1, 0.0);
        double tot = 0.0;
        for (int l = 0; l <= L; ++l) {
            yhat[l] = s1[l] / (double)done[l];
            var[l] = std::max(s2[l] / (double)done[l] - yhat[l] * yhat[l], 0.0);
            tot += std::sqrt(var[l] * cost(l));
        }
        rounds = round + 1;
        if (inexact) break;  // no N_l update from inexact or non-finite sums
        for (int l = 0; l <= L; ++l)
            N[l] = std::max<int64_t>(done[l], (int64_t)std::ceil(std::sqrt(var[l] / cost(l)) * 2.0 / (tol * tol) * tot));
        bool finished = false;
        if (std::fabs(yhat[L]) > bias_c && L < Lmax) {
            ++L;
            N.push_back(n_init);
            done.push_back(next_done);
            s1.push_back(next_s1);
            s2.push_back(next_s2);
        } else {
            bool need_more = false;
            for (int l = 0; l <= L; ++l) need_more |= N[l] > done[l];
            if (!need_more) {
                double v = 0.0;
                for (int l = 0; l <= L; ++l) v += var[l] / (double)done[l];
                converged = (std::fabs(yhat[L]) <= bias_c) && v <= tol * tol / 2.0 * (1 + 1e-12);
                finished = true;
            }
        }
        if (finished) break;
        if (max_rounds > 0 && rounds - start_round >= max_rounds) {
            paused = true;
            break;
        }
    }
    // nothing may still run on the buffers (a round that failed part-way has
    // not joined its queue streams)
    for (hipStream_t q : ctx->qstreams) (void)hipStreamSynchronize(q);
    (void)hipStreamSynchronize(st);
    if (hbuf) (void)hipHostFree(hbuf);
    if (rc < 0) return rc;
    if (state_out) {
        mlmc_estimate_state &S = *state_out;
        memset(&S, 0, sizeof S);
        S.L = L;
        S.rounds = rounds;
        for (int l = 0; l <= L; ++l) {
            S.N[l] = N[l];
            S.done[l] = done[l];
            S.s1[l] = s1[l];
            S.s2[l] = s2[l];
        }
        for (int l = 0; l <= Lmax; ++l) {
            S.n_promoted[l] = n_prom[l];
            S.n_noconv[l] = n_nc[l];
            S.dtype[l] = dts[l];
        }
        S.gpu_ms = gpu_ms;
        S.tol = tol;
        S.n_init = n_init;
        S.mixed = mixed;
        S.solver = (int32_t)solver;
        S.seed = c.seed;
    }
    // level means and variances from the sums (a level added in the last
    // round counts with the samples it has)
    yhat.assign(L + 1, 0.0);
    var.assign(L + 1, 0.0);
    for (int l = 0; l <= L; ++l)
        if (done[l] > 0) {
            yhat[l] = s1[l] / (double)done[l];
            var[l] = std::max(s2[l] / (double)done[l] - yhat[l] * yhat[l], 0.0);
        }
    memset(out, 0, sizeof *out);
    out->L = L;
    out->converged = converged;
    double est = 0.0, v = 0.0;
    double eps[16];
    mlmc_accuracy_targets(ctx, L, eps);
    for (int l = 0; l <= L; ++l) {
        est += yhat[l];
        v += done[l] > 0 ? var[l] / (double)done[l] : 0.0;
        out->N[l] = done[l];
        out->Yhat[l] = yhat[l];
        out->s2[l] = var[l];
        out->C[l] = cost(l);
        out->eps[l] = mixed ? eps[l] : std_eps;
    }
    for (int l = 0; l <= Lmax; ++l) {
        out->n_promoted[l] = n_prom[l];
        out->n_noconv[l] = n_nc[l];
    }
    out->estimate = est;
    out->var_est = v;
    out->gpu_ms = gpu_ms;
    out->wall_s = std::chrono::duration<double>(std::chrono::steady_clock::now() - t0).count();
    if (inexact) {
        out->converged = 0;
        fail(ctx, MLMC_ENOCONV, "estimate: samples missed their accuracy target or level sums are not finite");
        return MLMC_ENOCONV;
    }
    return paused ? MLMC_PAUSED : MLMC_OK;
}

int mlmc_mcmc(mlmc_ctx *ctx, const mlmc_mcmc_config *mc, mlmc_mcmc_result *out, void *stream)
{
    if (!ctx) return MLMC_EINVAL;
    if (!mc || !out) return fail(ctx, MLMC_EINVAL, "mcmc: null argument");
    const mlmc_config &c = ctx->cfg;
    if (mc->L < 0 || mc->L > c.L_max || mc->chains < 1 || mc->chains > 65536 || mc->burn_in < 0 ||
        mc->subsample < 1 || !(mc->pcn_beta > 0.0 && mc->pcn_beta <= 1.0) || !(mc->noise_sd > 0.0) ||
        mc->n_obs < 1 || mc->n_obs > 64)
        return fail(ctx, MLMC_EINVAL, "mcmc: bad configuration");
    int64_t total_steps = 0;
    for (int l = 0; l <= mc->L; ++l) {
        if (mc->steps[l] < 1) return fail(ctx, MLMC_EINVAL, "mcmc: steps[%d] < 1", l);
        const int64_t st_l = (int64_t)(mc->burn_in + mc->steps[l]) * (l > 0 ? mc->subsample : 1);
        if (st_l * mc->chains >= ((int64_t)1 << 32)) return fail(ctx, MLMC_EINVAL, "mcmc: too many draws");
        total_steps += mc->burn_in + mc->steps[l];
        if (int rc = check_opts(ctx, &mc->opts[l], l, true)) return rc;
    }
    // observation nodes: interior nodes of the level-0 grid
    int obs_node[64];
    for (int j = 0; j < mc->n_obs; ++j) {
        const double fx = mc->obs_x[j] * 1024.0, fy = mc->obs_y[j] * 1024.0;
        const double gx = mc->obs_x[j] * c.n0, gy = mc->obs_y[j] * c.n0;
        if (!(gx > 0.5 && gx < c.n0 - 0.5 && gy > 0.5 && gy < c.n0 - 0.5) || std::fabs(gx - std::round(gx)) > 1e-9 ||
            std::fabs(gy - std::round(gy)) > 1e-9 || !std::isfinite(mc->obs_value[j]))
            return fail(ctx, MLMC_EINVAL, "mcmc: observation %d is not an interior node of the coarsest grid", j);
        obs_node[j] = (int)std::lround(fx) + 1024 * (int)std::lround(fy);
    }
    const auto t0 = std::chrono::steady_clock::now();
    hipStream_t st = (hipStream_t)stream;
    const int C = mc->chains, K = c.K;
    // device buffers: states and proposals (C x K), per-chain scalars, the
    // solve workspaces of the finest level's two grids
    size_t need = 0;
    auto take = [&](size_t b) { size_t o = need; need += align256(b); return o; };
    const size_t o_obs = take(64 * 4), o_obsv = take(64 * 8);
    const size_t o_tf = take((size_t)C * K * 8), o_tc = take((size_t)C * K * 8), o_pr = take((size_t)C * K * 8),
                 o_w = take((size_t)C * K * 8), o_z = take((size_t)C * 8);
    const size_t o_llf = take(C * 8), o_llcf = take(C * 8), o_qf = take(C * 8), o_llc = take(C * 8),
                 o_qc = take(C * 8), o_qpf = take(C * 8), o_qpc = take(C * 8), o_dummy = take(C * 8);
    const size_t o_accf = take(C * 8), o_accc = take(C * 8), o_sums = take(2 * (size_t)C * 8);
    size_t wsf = 0, wsc = 0;
    for (int l = 0; l <= mc->L; ++l) {
        wsf = std::max(wsf, make_layout(c.n0 << l, C, mc->opts[l]).bytes);
        if (l > 0) wsc = std::max(wsc, make_layout(c.n0 << (l - 1), C, mc->opts[l]).bytes);
    }
    const size_t o_wsf = take(wsf), o_wsc = take(wsc);
    void *buf = nullptr;
    HIPCHK(hipMalloc(&buf, need));
    auto D = [&](size_t o) { return at<double>(buf, o); };
    int rc = MLMC_OK;
    std::vector<double> h_sums(2 * (size_t)C);
    std::vector<int64_t> h_acc(C);
    memset(out, 0, sizeof *out);
    int64_t solves = 0;
    double obs_v[64];
    for (int j = 0; j < mc->n_obs; ++j) obs_v[j] = mc->obs_value[j];
    const int *d_obs = at<int>(buf, o_obs);
    const double *d_obsv = D(o_obsv);
    auto run = [&]() -> int {
        HIPCHK(hipMemcpyAsync(at<int>(buf, o_obs), obs_node, mc->n_obs * 4, hipMemcpyHostToDevice, st));
        HIPCHK(hipMemcpyAsync(D(o_obsv), obs_v, mc->n_obs * 8, hipMemcpyHostToDevice, st));
        for (int l = 0; l <= mc->L; ++l) {
            const mlmc_level_opts &o = mc->opts[l];
            const int nf = c.n0 << l, nc = nf / 2;
            const grid_layout Lf = make_layout(nf, C, o);
            const grid_layout Lc = l > 0 ? make_layout(nc, C, o) : grid_layout{};
            void *wf = at<void>(buf, o_wsf), *wc = at<void>(buf, o_wsc);
            const uint32_t base = 4096 + 8 * (uint32_t)l;
            auto solve = [&](bool fine, const double *xi, double *q) -> int {
                ++solves;
                return fine ? solve_grid(ctx, Lf, l, xi, o, o.eps_fine, wf, q, at<int32_t>(wf, Lf.off_iters), st)
                            : solve_grid(ctx, Lc, l - 1, xi, o, o.eps_coarse, wc, q, at<int32_t>(wc, Lc.off_iters),
                                         st);
            };
            // start at xi = 0
            HIPCHK(hipMemsetAsync(D(o_tf), 0, (size_t)C * K * 8, st));
            HIPCHK(hipMemsetAsync(D(o_tc), 0, (size_t)C * K * 8, st));
            HIPCHK(hipMemsetAsync(D(o_accf), 0, (size_t)C * 8, st));
            HIPCHK(hipMemsetAsync(D(o_accc), 0, (size_t)C * 8, st));
            HIPCHK(hipMemsetAsync(D(o_sums), 0, 2 * (size_t)C * 8, st));
            if (int e = solve(true, D(o_tf), D(o_qf))) return e;
            HIPCHK(launch_mcmc_loglik(C, nf, mc->n_obs, d_obs, d_obsv, mc->noise_sd, at<double>(wf, Lf.off_x),
                                      D(o_llf), st));
            if (l > 0) {
                if (int e = solve(false, D(o_tc), D(o_qc))) return e;
                HIPCHK(launch_mcmc_loglik(C, nc, mc->n_obs, d_obs, d_obsv, mc->noise_sd, at<double>(wc, Lc.off_x),
                                          D(o_llc), st));
                HIPCHK(hipMemcpyAsync(D(o_llcf), D(o_llc), (size_t)C * 8, hipMemcpyDeviceToDevice, st));
            }
            const int nsteps = mc->burn_in + mc->steps[l];
            for (int k = 0; k < nsteps; ++k) {
                const int rec = k >= mc->burn_in;
                if (l == 0) {
                    HIPCHK(launch_fill_xi(mc->seed, base + 0, (int64_t)k * C, C, K, D(o_w), st));
                    HIPCHK(launch_pcn_propose(C, K, mc->pcn_beta, D(o_tf), D(o_w), D(o_pr), st));
                    if (int e = solve(true, D(o_pr), D(o_qpf))) return e;
                    HIPCHK(launch_fill_xi(mc->seed, base + 2, (int64_t)k * C, C, 1, D(o_z), st));
                    HIPCHK(launch_mcmc_accept(C, K, nf, 0, mc->n_obs, d_obs, d_obsv, mc->noise_sd,
                                              at<double>(wf, Lf.off_x), D(o_qpf), D(o_pr), D(o_dummy), D(o_z),
                                              D(o_tf), D(o_llf), D(o_dummy), D(o_qf), at<int64_t>(buf, o_accf), rec,
                                              st));
                    if (rec) HIPCHK(launch_mcmc_record(C, D(o_qf), nullptr, D(o_sums), st));
                    continue;
                }
                for (int sub = 0; sub < mc->subsample; ++sub) {
                    const int64_t idx = ((int64_t)k * mc->subsample + sub) * C;
                    HIPCHK(launch_fill_xi(mc->seed, base + 1, idx, C, K, D(o_w), st));
                    HIPCHK(launch_pcn_propose(C, K, mc->pcn_beta, D(o_tc), D(o_w), D(o_pr), st));
                    if (int e = solve(false, D(o_pr), D(o_qpc))) return e;
                    HIPCHK(launch_fill_xi(mc->seed, base + 3, idx, C, 1, D(o_z), st));
                    HIPCHK(launch_mcmc_accept(C, K, nc, 0, mc->n_obs, d_obs, d_obsv, mc->noise_sd,
                                              at<double>(wc, Lc.off_x), D(o_qpc), D(o_pr), D(o_dummy), D(o_z),
                                              D(o_tc), D(o_llc), D(o_dummy), D(o_qc), at<int64_t>(buf, o_accc), rec,
                                              st));
                }
                // the fine chain proposes the coarse chain's state
                HIPCHK(hipMemcpyAsync(D(o_pr), D(o_tc), (size_t)C * K * 8, hipMemcpyDeviceToDevice, st));
                if (int e = solve(true, D(o_pr), D(o_qpf))) return e;
                HIPCHK(launch_fill_xi(mc->seed, base + 2, (int64_t)k * C, C, 1, D(o_z), st));
                HIPCHK(launch_mcmc_accept(C, K, nf, 1, mc->n_obs, d_obs, d_obsv, mc->noise_sd,
                                          at<double>(wf, Lf.off_x), D(o_qpf), D(o_pr), D(o_llc), D(o_z), D(o_tf),
                                          D(o_llf), D(o_llcf), D(o_qf), at<int64_t>(buf, o_accf), rec, st));
                if (rec) HIPCHK(launch_mcmc_record(C, D(o_qf), D(o_qc), D(o_sums), st));
            }
            // level statistics: mean over chains and steps, variance of the mean
            // from the chain means (independent chains)
            HIPCHK(hipMemcpyAsync(h_sums.data(), D(o_sums), 2 * (size_t)C * 8, hipMemcpyDeviceToHost, st));
            HIPCHK(hipMemcpyAsync(h_acc.data(), D(o_accf), (size_t)C * 8, hipMemcpyDeviceToHost, st));
            HIPCHK(hipStreamSynchronize(st));
            const double T = (double)mc->steps[l];
            double mean = 0.0, acc = 0.0;
            for (int ch = 0; ch < C; ++ch) {
                mean += h_sums[2 * ch] / T;
                acc += (double)h_acc[ch];
            }
            mean /= C;
            double v = 0.0;
            for (int ch = 0; ch < C; ++ch) {
                const double d = h_sums[2 * ch] / T - mean;
                v += d * d;
            }
            out->Yhat[l] = mean;
            out->var_mean[l] = C > 1 ? v / ((double)C * (C - 1)) : 0.0;
            out->accept[l] = acc / ((double)C * T);
            if (l > 0) {
                HIPCHK(hipMemcpyAsync(h_acc.data(), D(o_accc), (size_t)C * 8, hipMemcpyDeviceToHost, st));
                HIPCHK(hipStreamSynchronize(st));
                double ac = 0.0;
                for (int ch = 0; ch < C; ++ch) ac += (double)h_acc[ch];
                out->accept_coarse[l] = ac / ((double)C * T * mc->subsample);
            }
            out->estimate += mean;
        }
        return MLMC_OK;
    };
    rc = run();
    (void)hipStreamSynchronize(st);
    (void)hipFree(buf);
    out->solves = solves;
    out->wall_s = std::chrono::duration<double>(std::chrono::steady_clock::now() - t0).count();
    (void)total_steps;
    return rc;
}

int mlmc_mimc(mlmc_ctx *ctx, const mlmc_mimc_config *mi, mlmc_mimc_result *out, void *stream)
{
    if (!ctx) return MLMC_EINVAL;
    if (!mi || !out) return fail(ctx, MLMC_EINVAL, "mimc: null argument");
    const mlmc_config &c = ctx->cfg;
    const int K = c.K, NI = mi->n_idx;
    if (NI < 1 || NI > 64 || mi->K0 < 1 || mi->K0 > K) return fail(ctx, MLMC_EINVAL, "mimc: bad configuration");
    for (int i = 0; i < NI; ++i) {
        const int l = mi->idx_l[i], k = mi->idx_k[i];
        if (l < 0 || l > c.L_max || k < 0 || k > 15 || mi->N[i] < 2 || mi->N[i] > ((int64_t)1 << 32))
            return fail(ctx, MLMC_EINVAL, "mimc: bad index %d", i);
        for (int j = 0; j < i; ++j)
            if (mi->idx_l[j] == l && mi->idx_k[j] == k) return fail(ctx, MLMC_EINVAL, "mimc: index %d repeated", i);
        if (int rc = check_opts(ctx, &mi->opts[i], l, true)) return rc;
    }
    const auto t0 = std::chrono::steady_clock::now();
    hipStream_t st = (hipStream_t)stream;
    if (int rc = ensure_queues(ctx, 2 + kQueues)) return rc;
    // Index i runs in chunks of Ci[i] samples whose fine and coarse solve
    // workspaces fit the budget; the indices are spread over the context's
    // queue streams (most expensive first onto the least loaded; cost
    // samples x n^3.5 x terms) and each stream runs its indices' chunks in
    // order in buffers of its own.  As in the multi-level step, the other
    // queues start when the most expensive index's first factorisation is
    // next in its queue.
    const size_t budget = (size_t)4 << 30;
    int64_t Ci[64], nch[64], sbase[64];
    int qof[64];
    double load[kQueues] = {};
    std::vector<int> order(NI);
    int64_t nsum = 0;
    for (int i = 0; i < NI; ++i) {
        const int l = mi->idx_l[i];
        // bytes per sample from a 4096-sample layout (the promotion pool is a
        // fraction of the batch)
        const size_t per = (make_layout(c.n0 << l, 4096, mi->opts[i]).bytes +
                            (l > 0 ? make_layout(c.n0 << (l - 1), 4096, mi->opts[i]).bytes : 0) + 4095) / 4096;
        Ci[i] = std::min<int64_t>({mi->N[i], (int64_t)1 << 20, std::max<int64_t>(1, (int64_t)(budget / per))});
        nch[i] = (mi->N[i] + Ci[i] - 1) / Ci[i];
        sbase[i] = nsum;
        nsum += nch[i];
        order[i] = i;
    }
    auto cost = [&](int i) {
        const double nn = (double)(c.n0 << mi->idx_l[i]);
        return (double)mi->N[i] * std::pow(nn, 3.5) * (mi->idx_l[i] ? 2 : 1) * (mi->idx_k[i] ? 2 : 1);
    };
    std::stable_sort(order.begin(), order.end(), [&](int a, int b) { return cost(a) > cost(b); });
    for (int i : order) {
        int q = 0;
        for (int t = 1; t < kQueues; ++t)
            if (load[t] < load[q]) q = t;
        qof[i] = q;
        load[q] += cost(i);
    }
    // per queue: the largest chunk and workspaces of its indices
    struct qbuf { int64_t C = 0; size_t wsf = 0, wsc = 0, o_xi, o_xm, o_y, o_sy, o_q[4], o_s[4], o_wsf, o_wsc; };
    qbuf Q[kQueues];
    for (int i = 0; i < NI; ++i) {
        const int l = mi->idx_l[i];
        qbuf &B = Q[qof[i]];
        B.C = std::max(B.C, Ci[i]);
        B.wsf = std::max(B.wsf, make_layout(c.n0 << l, Ci[i], mi->opts[i]).bytes);
        if (l > 0) B.wsc = std::max(B.wsc, make_layout(c.n0 << (l - 1), Ci[i], mi->opts[i]).bytes);
    }
    size_t need = 0;
    auto take = [&](size_t b) { size_t o = need; need += align256(std::max<size_t>(b, 1)); return o; };
    const size_t o_sums = take((size_t)nsum * 8 * 8);
    for (int q = 0; q < kQueues; ++q) {
        qbuf &B = Q[q];
        if (B.C == 0) continue;
        B.o_xi = take((size_t)B.C * K * 8);
        B.o_xm = take((size_t)B.C * K * 8);
        B.o_y = take((size_t)B.C * 8);
        B.o_sy = take((size_t)B.C * 4);
        for (int e = 0; e < 4; ++e) {
            B.o_q[e] = take((size_t)B.C * 8);
            B.o_s[e] = take((size_t)B.C * 4);
        }
        B.o_wsf = take(B.wsf);
        B.o_wsc = take(B.wsc);
    }
    void *buf = nullptr;
    HIPCHK(hipMalloc(&buf, need));
    memset(out, 0, sizeof *out);
    int64_t solves = 0;
    std::vector<double> h((size_t)nsum * 8);
    auto run = [&]() -> int {
        hipEvent_t fork = ctx->qevents[0], head = ctx->qevents[1 + kQueues];
        HIPCHK(hipEventRecord(fork, st));
        const int q0 = qof[order[0]];
        HIPCHK(hipStreamWaitEvent(ctx->qstreams[q0], fork, 0));
        bool gated = false;
        for (int i : order) {
            const int l = mi->idx_l[i], k = mi->idx_k[i];
            const mlmc_level_opts &o = mi->opts[i];
            const int nf = c.n0 << l;
            const qbuf &B = Q[qof[i]];
            hipStream_t sq = ctx->qstreams[qof[i]];
            for (int64_t ch = 0; ch < nch[i]; ++ch) {
                const int64_t first = ch * Ci[i], cc = std::min(Ci[i], mi->N[i] - first);
                const grid_layout Lf = make_layout(nf, cc, o);
                const grid_layout Lc = l > 0 ? make_layout(nf / 2, cc, o) : grid_layout{};
                void *wf = at<void>(buf, B.o_wsf), *wc = at<void>(buf, B.o_wsc);
                HIPCHK(launch_fill_xi(mi->seed, 8192 + i, first, cc, K, at<double>(buf, B.o_xi), sq));
                // term e = 2 t + g: truncation t (0: K_k, 1: K_{k-1}), grid g (0: l, 1: l - 1)
                bool have[4] = {false, false, false, false};
                for (int t = 0; t < (k > 0 ? 2 : 1); ++t) {
                    const int64_t keep = std::min<int64_t>(K, (int64_t)mi->K0 << (k - t));
                    HIPCHK(launch_mask_modes((int)cc, K, (int)keep, at<double>(buf, B.o_xi), at<double>(buf, B.o_xm),
                                             sq));
                    for (int g = 0; g < (l > 0 ? 2 : 1); ++g) {
                        const int e = 2 * t + g;
                        const grid_layout &G = g ? Lc : Lf;
                        void *w = g ? wc : wf;
                        ++solves;
                        if (int rc = solve_grid(ctx, G, l - g, at<double>(buf, B.o_xm), o,
                                                g ? o.eps_coarse : o.eps_fine, w, at<double>(buf, B.o_q[e]),
                                                at<int32_t>(w, G.off_iters), sq, gated ? nullptr : head))
                            return rc;
                        if (!gated) {
                            gated = true;
                            for (int q = 0; q < kQueues; ++q)
                                if (q != q0 && Q[q].C) HIPCHK(hipStreamWaitEvent(ctx->qstreams[q], head, 0));
                        }
                        HIPCHK(hipMemcpyAsync(at<uint32_t>(buf, B.o_s[e]), at<uint32_t>(w, G.off_state),
                                              (size_t)cc * 4, hipMemcpyDeviceToDevice, sq));
                        have[e] = true;
                    }
                }
                auto Qe = [&](int e) { return have[e] ? at<double>(buf, B.o_q[e]) : nullptr; };
                auto Se = [&](int e) { return have[e] ? at<uint32_t>(buf, B.o_s[e]) : nullptr; };
                HIPCHK(launch_mimc_combine((int)cc, Qe(0), Qe(1), Qe(2), Qe(3), Se(0), Se(1), Se(2), Se(3),
                                           at<double>(buf, B.o_y), at<uint32_t>(buf, B.o_sy), sq));
                HIPCHK(launch_pair_sums((int)cc, at<double>(buf, B.o_y), nullptr, at<uint32_t>(buf, B.o_sy), nullptr,
                                        nullptr, nullptr, nullptr, nullptr,
                                        at<double>(buf, o_sums) + (size_t)(sbase[i] + ch) * 8, sq));
            }
        }
        for (int q = 0; q < kQueues; ++q) {
            if (!Q[q].C) continue;
            HIPCHK(hipEventRecord(ctx->qevents[1 + q], ctx->qstreams[q]));
            HIPCHK(hipStreamWaitEvent(st, ctx->qevents[1 + q], 0));
        }
        HIPCHK(hipMemcpyAsync(h.data(), at<double>(buf, o_sums), (size_t)nsum * 8 * 8, hipMemcpyDeviceToHost, st));
        HIPCHK(hipStreamSynchronize(st));
        for (int i = 0; i < NI; ++i) {
            // chunk sums added in chunk order (fixed order)
            double sy = 0.0, sy2 = 0.0;
            int64_t npro = 0, nnc = 0;
            for (int64_t ch = 0; ch < nch[i]; ++ch) {
                const double *hh = &h[(size_t)(sbase[i] + ch) * 8];
                sy += hh[0];
                sy2 += hh[1];
                npro += (int64_t)hh[4];
                nnc += (int64_t)hh[5];
            }
            const double N = (double)mi->N[i], mean = sy / N;
            out->mean[i] = mean;
            out->var[i] = std::max(0.0, (sy2 - N * mean * mean) / (N - 1.0));
            out->n_promoted[i] = npro;
            out->n_noconv[i] = nnc;
            out->estimate += mean;
            out->var_estimate += out->var[i] / N;
        }
        return MLMC_OK;
    };
    int rc = run();
    for (hipStream_t q : ctx->qstreams) (void)hipStreamSynchronize(q);
    (void)hipStreamSynchronize(st);
    (void)hipFree(buf);
    out->solves = solves;
    out->wall_s = std::chrono::duration<double>(std::chrono::steady_clock::now() - t0).count();
    if (rc) return rc;
    for (int i = 0; i < NI; ++i)
        if (out->n_noconv[i] > 0) return fail(ctx, MLMC_ENOCONV, "mimc: index %d has %lld non-converged samples", i,
                                              (long long)out->n_noconv[i]);
    return MLMC_OK;
}

int mlmc_profile(mlmc_ctx *ctx, int32_t enable)
{
    if (!ctx) return MLMC_EINVAL;
    for (auto &r : ctx->prof) {
        ctx->ev_pool.push_back(r.a);
        ctx->ev_pool.push_back(r.b);
    }
    ctx->prof.clear();
    ctx->prof_on = enable != 0;
    return MLMC_OK;
}

int mlmc_profile_read(mlmc_ctx *ctx, int32_t kind, int32_t n, double *total_ms, int64_t *launches,
                      int64_t *samples)
{
    if (!ctx || !total_ms || !launches || !samples) return MLMC_EINVAL;
    double ms = 0.0;
    int64_t cnt = 0, smp = 0;
    for (auto &r : ctx->prof) {
        if (r.kind != kind || r.n != n) continue;
        HIPCHK(hipEventSynchronize(r.b));
        float t = 0.f;
        HIPCHK(hipEventElapsedTime(&t, r.a, r.b));
        ms += t;
        ++cnt;
        smp += r.samples;
    }
    *total_ms = ms;
    *launches = cnt;
    *samples = smp;
    return MLMC_OK;
}

int mlmc_grad(mlmc_ctx *ctx, int32_t level, int64_t n, const double *xi_dev, const double *grad_q_dev,
              const mlmc_level_opts *opts, double eps_adjoint, void *ws_dev, size_t ws_bytes,
              double *grad_xi_dev, void *stream)
{
    int rc = check_level(ctx, level);
    if (rc) return rc;
    if ((rc = check_opts(ctx, opts, level, false))) return rc;
    if (is_iterative(opts->solver)) return fail(ctx, MLMC_EINVAL, "grad needs a factorisation (not an iterative solver)");
    if (n < 0 || n > 4000000) return fail(ctx, MLMC_EINVAL, "bad sample count (0..4e6)");
    if (n == 0) return MLMC_OK;
    if (!xi_dev || !ws_dev || !grad_xi_dev || !(eps_adjoint > 0.0) || !aligned(xi_dev, 8) ||
        !aligned(grad_q_dev, 8) || !aligned(grad_xi_dev, 8))
        return fail(ctx, MLMC_EINVAL, "grad: bad arguments");
    if (((uintptr_t)ws_dev & 255) != 0) return fail(ctx, MLMC_EINVAL, "workspace not 256-byte aligned");
    const level_layout LL = make_level_layout(ctx->cfg, level, n, *opts);
    if (ws_bytes < LL.bytes) return fail(ctx, MLMC_ENOMEM, "workspace %zu < %zu bytes", ws_bytes, LL.bytes);
    hipStream_t st = (hipStream_t)stream;
    const grid_layout &L = LL.fine;
    void *ws = at<void>(ws_dev, LL.off_fine);
    const int S = (int)n, nn = L.n, K = ctx->cfg.K, P = (nn + 1) * (nn + 1);
    const bool direct = opts->solver == MLMC_DIRECT;
    const int dt = direct ? MLMC_F64 : opts->factor_dtype;
    // adjoint state: A lambda = dQ/du = h^2 1 (rhs with fconst = 1), refined in FP64
    HIPCHK(launch_init_state(S, at<uint32_t>(ws, L.off_state), at<double>(ws, L.off_relres), st));
    double *lam = at<double>(ws, L.off_lam);
    rc = refine(ctx, L, ws, dt, false, 1.0, eps_adjoint, lam, at<double>(ws, L.off_q), nullptr, st);
    if (rc) return rc;
    double *gz = at<double>(ws, L.off_gz);
    HIPCHK(launch_adjoint_gz(nn, S, at<double>(ws, L.off_a), at<double>(ws, L.off_x), lam, gz, ctx->cfg.disc,
                             st));
    HIPCHK(launch_grad_gemm(S, K, P, gz, ctx->phit[level], grad_q_dev, grad_xi_dev, st));
    return MLMC_OK;
}

}  // extern "C"

