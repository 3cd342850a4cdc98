// qs_prob_noalloc: the probability reduction of qs_calc_total_prob /
// qs_calc_prob_of_outcome over caller-owned amplitudes, for callers that
// cannot allocate device memory (code under HIP graph capture, serving loops
// that must not call hipMalloc).  A register handle would bring its own
// reduction partials (allocated at qs_reg_create / qs_reg_wrap); here the
// partials live in one file-scope device array per GPU, `scratch`, whose
// device address is looked up once per device with hipGetSymbolAddress.  The
// host never passes the array's name to a kernel: only the looked-up
// address.
#include <mutex>
#include <string>

#include "qs_host.h"
#include "qstate_noalloc.h"

namespace {

// Reduction partials: 2 compensated sums (value, compensation) per block,
// at most kReduceBlocks blocks.  Each block writes its own four doubles
// before the final fold reads them, so nothing needs clearing between calls.
constexpr size_t kNoAllocScratchDoubles = 4 * qs::kReduceBlocks;
static __device__ __align__(256) double scratch[kNoAllocScratchDoubles];

constexpr int kMaxDevices = 64;
std::mutex g_mu;
double* g_ptr[kMaxDevices] = {};  // device address of `scratch` per device

// Address of this device's copy of `scratch`; `device` must be current.
qs_status scratch_ptr(int device, double** out)
{
    std::lock_guard<std::mutex> g(g_mu);
    if (!g_ptr[device]) {
        void* p = nullptr;
        const hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
        if (e != hipSuccess || !p) return qs::hip_error(e != hipSuccess ? e : hipErrorInvalidSymbol, "hipGetSymbolAddress");
        g_ptr[device] = (double*)p;
    }
    *out = g_ptr[device];
    return QS_OK;
}

}  // namespace

extern "C" {

qs_status qs_prob_noalloc(int device, const void* dev_amps, int n, int kind, int prec, int qubit, double* dev_out,
                          void* hip_stream)
{
    if (!dev_amps || !dev_out) return qs::set_error(QS_E_ARG, "NULL device pointer");
    if (kind != QS_STATEVEC && kind != QS_DENSITY) return qs::set_error(QS_E_ARG, "unknown register kind");
    if (prec != QS_C64 && prec != QS_C128) return qs::set_error(QS_E_ARG, "unknown precision");
    const int nmax = kind == QS_DENSITY ? 20 : 40;
    if (n < 1 || n > nmax)
        return qs::set_error(QS_E_ARG, "qubit count outside [1, " + std::to_string(nmax) + "]");
    if (qubit < -1 || qubit >= n) return qs::set_error(QS_E_ARG, "qubit outside [-1, n)");
    int count = 0;
    hipError_t e = hipGetDeviceCount(&count);
    if (e != hipSuccess) return qs::hip_error(e, "hipGetDeviceCount");
    if (device < 0 || device >= count || device >= kMaxDevices) return qs::set_error(QS_E_ARG, "invalid device");
    e = hipSetDevice(device);
    if (e != hipSuccess) return qs::hip_error(e, "hipSetDevice");
    double* partials = nullptr;
    qs_status s = scratch_ptr(device, &partials);
    if (s) return s;
    // every launch below uses at most kReduceBlocks blocks, 4 partials each
    const qs::Launch L{(hipStream_t)hip_stream, device};
    if (kind == QS_DENSITY)
        e = prec == QS_C128 ? qs::launch_prob_dm<double>(L, dev_amps, n, qubit, partials, dev_out)
                            : qs::launch_prob_dm<float>(L, dev_amps, n, qubit, partials, dev_out);
    else
        e = prec == QS_C128 ? qs::launch_prob_sv<double>(L, dev_amps, n, qubit, partials, dev_out)
                            : qs::launch_prob_sv<float>(L, dev_amps, n, qubit, partials, dev_out);
    if (e != hipSuccess) return qs::hip_error(e, "kernel launch");
    return QS_OK;
}

}  // extern "C"
