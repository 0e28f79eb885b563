// Stub HIP runtime for host-only checks of the library's host logic (no GPU):
// allocations are host memory, launches and synchronisations return at once,
// device-to-host copies of a chunk's eight level sums deliver 0.5 in every
// sum slot, 0 promoted and (STUB_NOCONV set in the environment) one
// non-converged sample, so that the estimator's level test adds levels or
// its non-convergence path runs; an event query reports "not ready" two
// times in three (the estimator's polling path).  The launchers of the device
// kernels do no work; factor_entries_per_sample restates the library's
// workspace sizing for the layout code that calls it.
//
// Capture model: between hipStreamBeginCapture and hipStreamEndCapture every
// operation is checked against the rules of stream capture: a launch, copy or
// record on a stream outside the capture, a wait on an event that was not
// recorded inside the capture, or a synchronisation inside the capture
// aborts; at the end every stream that joined the capture (through a wait on
// a captured event) must be joined back to the origin stream, directly or
// through other captured streams, after its last operation.
#include <hip/hip_runtime_api.h>
#include <cstdint>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <map>
#include <set>
#include <vector>
#include "kernels.h"  // the library's internal launcher declarations

namespace {
[[noreturn]] void die(const char *what)
{
    fprintf(stderr, "stub runtime: %s\n", what);
    abort();
}

struct rec_t { hipStream_t s; long pos; long epoch; };
struct edge_t { hipStream_t src; long pos; hipStream_t dst; long at; };

std::map<hipStream_t, long> g_ops;   // operations enqueued per stream
std::map<hipEvent_t, rec_t> g_rec;   // last record of every event
bool g_capturing = false;
long g_epoch = 0;
hipStream_t g_origin = nullptr;
std::set<hipStream_t> g_cap;         // streams inside the capture
std::vector<edge_t> g_edges;         // captured waits

hipError_t op(hipStream_t s)
{
    if (g_capturing && !g_cap.count(s)) die("operation on a stream outside the capture");
    ++g_ops[s];
    return hipSuccess;
}

void no_sync(hipStream_t s)
{
    if (g_capturing && (s == nullptr || g_cap.count(s))) die("synchronisation inside a capture");
}

// Whether the operations of s up to position pos reach the origin's end.
bool covered(hipStream_t s, long pos, int depth)
{
    if (s == g_origin) return true;
    if (depth > 64) die("capture dependency chain too deep");
    for (const edge_t &e : g_edges)
        if (e.src == s && e.pos >= pos && covered(e.dst, e.at, depth + 1)) return true;
    return false;
}

int g_obj[4096];
int g_next = 0;
void *newobj() { return &g_obj[(g_next++) % 4096]; }
int g_q = 0;
}  // namespace

extern "C" {
hipError_t hipMalloc(void **p, size_t n) { *p = aligned_alloc(256, (n + 255) & ~(size_t)255); return *p ? hipSuccess : hipErrorOutOfMemory; }
hipError_t hipFree(void *p) { free(p); return hipSuccess; }
hipError_t hipMemsetAsync(void *, int, size_t, hipStream_t st) { return op(st); }
hipError_t hipHostMalloc(void **p, size_t n, unsigned int) { *p = malloc(n); return hipSuccess; }
hipError_t hipHostFree(void *p) { free(p); return hipSuccess; }
hipError_t hipMemcpy(void *d, const void *s, size_t n, hipMemcpyKind)
{
    if (g_capturing) die("synchronous copy inside a capture");
    memmove(d, s, n);
    return hipSuccess;
}
hipError_t hipMemcpyAsync(void *d, const void *s, size_t n, hipMemcpyKind k, hipStream_t st)
{
    (void)op(st);
    if (k == hipMemcpyDeviceToHost) {
        const double noconv = getenv("STUB_NOCONV") ? 1.0 : 0.0;
        for (size_t q = 0; q + 8 <= n; q += 8) {
            const size_t slot = (q / 8) % 8;  // sum_y sum_y2 sum_qf sum_qc promoted noconv iters iters
            const double v = slot == 4 ? 0.0 : (slot == 5 ? noconv : 0.5);
            memcpy((char *)d + q, &v, 8);
        }
    } else {
        memmove(d, s, n);
    }
    return hipSuccess;
}
hipError_t hipStreamCreateWithFlags(hipStream_t *s, unsigned int) { *s = (hipStream_t)newobj(); return hipSuccess; }
hipError_t hipStreamDestroy(hipStream_t) { return hipSuccess; }
hipError_t hipStreamSynchronize(hipStream_t s) { no_sync(s); return hipSuccess; }
hipError_t hipStreamWaitEvent(hipStream_t s, hipEvent_t e, unsigned int)
{
    if (!e) die("wait on null event");
    auto it = g_rec.find(e);
    if (g_capturing) {
        const bool in_cap = it != g_rec.end() && it->second.epoch == g_epoch;
        if (!in_cap) die("wait inside a capture on an event not recorded in it");
        g_cap.insert(s);  // the waiting stream joins the capture
        g_edges.push_back({it->second.s, it->second.pos, s, g_ops[s]});
    } else if (it == g_rec.end()) {
        die("wait on an event that was never recorded");
    }
    return hipSuccess;
}
hipError_t hipStreamBeginCapture(hipStream_t s, hipStreamCaptureMode)
{
    if (g_capturing) die("nested capture");
    if (s == nullptr) die("capture of the null stream");
    g_capturing = true;
    ++g_epoch;
    g_origin = s;
    g_cap = {s};
    g_edges.clear();
    return hipSuccess;
}
hipError_t hipStreamEndCapture(hipStream_t s, hipGraph_t *g)
{
    if (!g_capturing || s != g_origin) die("end of a capture that was not begun on this stream");
    for (hipStream_t t : g_cap)
        if (t != g_origin && !covered(t, g_ops[t], 0)) die("a forked stream is not joined back to the origin");
    g_capturing = false;
    g_cap.clear();
    *g = (hipGraph_t)newobj();
    return hipSuccess;
}
hipError_t hipEventCreate(hipEvent_t *e) { *e = (hipEvent_t)newobj(); return hipSuccess; }
hipError_t hipEventCreateWithFlags(hipEvent_t *e, unsigned) { *e = (hipEvent_t)newobj(); return hipSuccess; }
hipError_t hipEventDestroy(hipEvent_t) { return hipSuccess; }
hipError_t hipEventRecord(hipEvent_t e, hipStream_t s)
{
    if (!e) die("record of null event");
    if (g_capturing && !g_cap.count(s)) die("record on a stream outside the capture");
    g_rec[e] = {s, g_ops[s], g_capturing ? g_epoch : 0};
    return hipSuccess;
}
hipError_t hipEventSynchronize(hipEvent_t e)
{
    auto it = g_rec.find(e);
    if (it != g_rec.end() && it->second.epoch == g_epoch && g_capturing) die("event synchronisation inside a capture");
    return hipSuccess;
}
hipError_t hipEventQuery(hipEvent_t e) { if (!e) abort(); if (g_capturing) die("event query inside a capture"); return (++g_q % 3) ? hipErrorNotReady : hipSuccess; }
hipError_t hipEventElapsedTime(float *ms, hipEvent_t, hipEvent_t) { *ms = 1.f; return hipSuccess; }
hipError_t hipGraphInstantiate(hipGraphExec_t *x, hipGraph_t, hipGraphNode_t *, char *, size_t) { *x = (hipGraphExec_t)newobj(); return hipSuccess; }
hipError_t hipGraphLaunch(hipGraphExec_t, hipStream_t s) { return op(s); }
hipError_t hipGraphDestroy(hipGraph_t) { return hipSuccess; }
hipError_t hipGraphExecDestroy(hipGraphExec_t) { return hipSuccess; }
const char *hipGetErrorString(hipError_t) { return "stub"; }
hipError_t hipGetDevice(int *d) { *d = 0; return hipSuccess; }
}
namespace mlmc {
size_t factor_entries_per_sample(int dtype, int n)
{
    if (use_blk(dtype, n)) { const int NB = n / 16; return (size_t)(n - 1) * (NB * (NB + 1) / 2) * 256; }
    int TR = n <= 16 ? 2 : (n <= 32 ? 4 : 8); const int Tn = n / TR, T = Tn * (Tn + 1) / 2;
    return (size_t)(n - 1) * T * TR * TR;
}
// the scratch array's device address: a fake address (the stub launchers never touch memory)
hipError_t scratch_device_ptr(int, void **out) { *out = (void *)(uintptr_t)0x200000000ull; return hipSuccess; }
hipError_t launch_fill_xi(uint64_t, int, int64_t, int64_t, int, double *, hipStream_t st) { return op(st); }
hipError_t launch_field(int, int, int, const double *, const double *, double *, hipStream_t st) { return op(st); }
hipError_t launch_grad_gemm(int, int, int, const double *, const double *, const double *, double *, hipStream_t st) { return op(st); }
hipError_t launch_coeffs(int, int, const double *, double *, double *, double *, int, hipStream_t st) { return op(st); }
hipError_t launch_factor(int, int, int, const double *, double *, double *, const double *, void *, const int *, const int *, int64_t, uint32_t *, double, double *, double *, int, int, hipStream_t st) { return op(st); }
bool factor_fuses_forward(int dtype, int n) { return use_blk(dtype, n) && (dtype != 0 || n == 16); }
bool factor_solves_initial(int dtype, int n) { return n == 16 || (factor_fuses_forward(dtype, n) && n <= 128); }
hipError_t launch_ir(int, const ir_args &, hipStream_t st) { return op(st); }
hipError_t launch_minres(int, int, double, const double *, const double *, const double *, const double *, double *, double *, void *, int, double, int, int, const int *, const int *, uint32_t *, double *, double *, int32_t *, int, hipStream_t st) { return op(st); }
hipError_t launch_adjoint_gz(int, int, const double *, const double *, const double *, double *, int, hipStream_t st) { return op(st); }
hipError_t launch_pcn_propose(int, int, double, const double *, const double *, double *, hipStream_t st) { return op(st); }
hipError_t launch_mcmc_accept(int, int, int, int, int, const int *, const double *, double, const double *, const double *, const double *, const double *, const double *, double *, double *, double *, double *, int64_t *, int, hipStream_t st) { return op(st); }
hipError_t launch_mcmc_loglik(int, int, int, const int *, const double *, double, const double *, double *, hipStream_t st) { return op(st); }
hipError_t launch_mcmc_record(int, const double *, const double *, double *, hipStream_t st) { return op(st); }
hipError_t launch_mask_modes(int, int, int, const double *, double *, hipStream_t st) { return op(st); }
hipError_t launch_mimc_combine(int, const double *, const double *, const double *, const double *, const uint32_t *, const uint32_t *, const uint32_t *, const uint32_t *, double *, uint32_t *, hipStream_t st) { return op(st); }
size_t mgcg_floats_per_sample(int n) { size_t t = 0; for (int l = 0; (n >> l) >= 2; ++l) { const size_t nl = n >> l, np = nl + 1; t += 2 * np * nl + 3 * np * np; } return (t + 63) & ~(size_t)63; }
hipError_t launch_mgcg(int, int, double, const double *, double *, double *, float *, double, int, uint32_t *, double *, double *, int32_t *, int, hipStream_t st) { return op(st); }
hipError_t launch_unpad(int, int, const double *, double *, hipStream_t st) { return op(st); }
hipError_t launch_init_state(int, uint32_t *, double *, hipStream_t st) { return op(st); }
hipError_t launch_reset_subset(int, const int *, const int *, uint32_t *, double *, hipStream_t st) { return op(st); }
hipError_t launch_zero_int(int *, int, hipStream_t st) { return op(st); }
hipError_t launch_collect(int, const uint32_t *, int *, int *, hipStream_t st) { return op(st); }
hipError_t launch_pair_sums(int, const double *, const double *, const uint32_t *, const uint32_t *, const int32_t *, const int32_t *, double *, uint8_t *, double *, hipStream_t st) { return op(st); }
}
