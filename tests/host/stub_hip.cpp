// Stub HIP runtime for host-only checks of the library's host logic (no GPU):
// allocations are host memory, launches and synchronisations return at once,
// device-to-host copies deliver 0.5 in every double (so that the estimator's
// level test adds levels), and an event query reports "not ready" two times
// in three (the estimator's polling path).  The launchers of the device
// kernels are no-ops; factor_entries_per_sample restates the library's
// workspace sizing for the layout code that calls it.
#include <hip/hip_runtime_api.h>
#include <cstdlib>
#include <cstring>
#include <cstdio>
#include "kernels.h"  // the library's internal launcher declarations
extern "C" {
hipError_t hipMalloc(void **p, size_t n) { *p = aligned_alloc(256, (n + 255) & ~(size_t)255); return *p ? hipSuccess : hipErrorOutOfMemory; }
hipError_t hipFree(void *p) { free(p); return hipSuccess; }
hipError_t hipHostMalloc(void **p, size_t n, unsigned int) { *p = malloc(n); return hipSuccess; }
hipError_t hipHostFree(void *p) { free(p); return hipSuccess; }
hipError_t hipMemcpy(void *d, const void *s, size_t n, hipMemcpyKind) { memmove(d, s, n); return hipSuccess; }
hipError_t hipMemcpyAsync(void *d, const void *s, size_t n, hipMemcpyKind k, hipStream_t) { if (k == hipMemcpyDeviceToHost) { for (size_t q = 0; q + 8 <= n; q += 8) { const double v = 0.5; memcpy((char *)d + q, &v, 8); } } else memmove(d, s, n); return hipSuccess; }
static int g_obj[4096]; static int g_next = 0;
static void *newobj() { return &g_obj[(g_next++) % 4096]; }
hipError_t hipStreamCreateWithFlags(hipStream_t *s, unsigned int) { *s = (hipStream_t)newobj(); return hipSuccess; }
hipError_t hipStreamDestroy(hipStream_t) { return hipSuccess; }
hipError_t hipStreamSynchronize(hipStream_t) { return hipSuccess; }
hipError_t hipStreamWaitEvent(hipStream_t, hipEvent_t e, unsigned int) { if (!e) { fprintf(stderr, "wait on null event\n"); abort(); } return hipSuccess; }
hipError_t hipStreamBeginCapture(hipStream_t, hipStreamCaptureMode) { return hipSuccess; }
hipError_t hipStreamEndCapture(hipStream_t, hipGraph_t *g) { *g = (hipGraph_t)newobj(); return hipSuccess; }
hipError_t hipEventCreate(hipEvent_t *e) { *e = (hipEvent_t)newobj(); return hipSuccess; }
hipError_t hipEventCreateWithFlags(hipEvent_t *e, unsigned) { *e = (hipEvent_t)newobj(); return hipSuccess; }
hipError_t hipEventDestroy(hipEvent_t) { return hipSuccess; }
hipError_t hipEventRecord(hipEvent_t e, hipStream_t) { if (!e) { fprintf(stderr, "record of null event\n"); abort(); } return hipSuccess; }
hipError_t hipEventSynchronize(hipEvent_t) { return hipSuccess; }
static int g_q = 0;
hipError_t hipEventQuery(hipEvent_t e) { if (!e) abort(); return (++g_q % 3) ? hipErrorNotReady : hipSuccess; }
hipError_t hipEventElapsedTime(float *ms, hipEvent_t, hipEvent_t) { *ms = 1.f; return hipSuccess; }
hipError_t hipGraphInstantiate(hipGraphExec_t *x, hipGraph_t, hipGraphNode_t *, char *, size_t) { *x = (hipGraphExec_t)newobj(); return hipSuccess; }
hipError_t hipGraphLaunch(hipGraphExec_t, hipStream_t) { return hipSuccess; }
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
#define ST(...) { return hipSuccess; }
hipError_t launch_fill_xi(uint64_t, int, int64_t, int64_t, int, double *, hipStream_t) ST()
hipError_t launch_field(int, int, int, const double *, const double *, double *, hipStream_t) ST()
hipError_t launch_grad_gemm(int, int, int, const double *, const double *, const double *, double *, hipStream_t) ST()
hipError_t launch_coeffs(int, int, const double *, double *, double *, double *, hipStream_t) ST()
hipError_t launch_factor(int, int, int, const double *, double *, double *, const double *, void *, const int *, const int *, int64_t, uint32_t *, double, double *, double *, hipStream_t) ST()
bool factor_fuses_forward(int dtype, int n) { return use_blk(dtype, n) && (dtype != 0 || n == 16); }
hipError_t launch_ir(int, const ir_args &, hipStream_t) ST()
hipError_t launch_minres(int, int, double, const double *, const double *, const double *, const double *, double *, double *, double *, double, int, uint32_t *, double *, double *, int32_t *, hipStream_t) ST()
hipError_t launch_adjoint_gz(int, int, const double *, const double *, const double *, double *, hipStream_t) ST()
hipError_t launch_unpad(int, int, const double *, double *, hipStream_t) ST()
hipError_t launch_init_state(int, uint32_t *, double *, hipStream_t) ST()
hipError_t launch_reset_subset(int, const int *, const int *, uint32_t *, double *, hipStream_t) ST()
hipError_t launch_zero_int(int *, int, hipStream_t) ST()
hipError_t launch_collect(int, const uint32_t *, int *, int *, hipStream_t) ST()
hipError_t launch_pair_sums(int, const double *, const double *, const uint32_t *, const uint32_t *, const int32_t *, const int32_t *, double *, uint8_t *, double *, hipStream_t) ST()
}
