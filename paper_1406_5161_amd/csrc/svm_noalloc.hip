// svm_noalloc.hip -- the classifier of eq:classi for callers that cannot allocate device
// memory: svm_decision's kernels on a scratch array that the library holds in each GPU's
// memory from the first call on that GPU until the process ends.
#include <hip/hip_runtime.h>

#include <mutex>

#include "svm_internal.h"

namespace {

constexpr size_t NOALLOC_SCRATCH_BYTES = 96ull << 20;   // 96 MiB per GPU
constexpr int MAX_DEVICES = 64;

// One copy per GPU that loads the library; on the host this name only stands for the symbol,
// the device address comes from hipGetSymbolAddress.
static __device__ __align__(256) unsigned char scratch[NOALLOC_SCRATCH_BYTES];

std::mutex g_mu;
void* g_scratch[MAX_DEVICES] = {};

// The current device's copy of the scratch array (looked up once per device).
int scratch_on_current_device(void** out) {
    int dev = 0;
    hipError_t e = hipGetDevice(&dev);
    if (e != hipSuccess) { svm::set_last_hip_error(e); return SVM_EHIP; }
    if (dev < 0 || dev >= MAX_DEVICES) return SVM_EUNSUPPORTED;
    std::lock_guard<std::mutex> lock(g_mu);
    if (!g_scratch[dev]) {
        void* p = nullptr;
        e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
        if (e != hipSuccess || !p) {
            svm::set_last_hip_error(e != hipSuccess ? e : hipErrorInvalidSymbol);
            return SVM_EHIP;
        }
        g_scratch[dev] = p;
    }
    *out = g_scratch[dev];
    return SVM_OK;
}

}  // namespace

extern "C" int svm_decision_noalloc(const svm_problem_t* train, const double* alpha, double beta, double gamma,
                                    const svm_problem_t* queries, double* out, int32_t kernel_precision,
                                    void* stream) {
    void* ws = nullptr;
    int rc = scratch_on_current_device(&ws);
    if (rc) return rc;
    size_t need = 0;
    rc = svm::decision_in_workspace(train, alpha, beta, gamma, queries, out, kernel_precision, ws,
                                    NOALLOC_SCRATCH_BYTES, (hipStream_t)stream, &need);
    return rc == SVM_EWORKSPACE && need > NOALLOC_SCRATCH_BYTES ? SVM_ESCRATCH : rc;
}
