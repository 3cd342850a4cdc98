// The qstate C ABI: handle management, host-side validation and dispatch to
// the gfx950 kernels.  Validation always completes before the first launch,
// so a call that fails leaves the register as it was.
#include <math.h>
#include <stdio.h>
#include <stdlib.h>
#include <string.h>

#include <algorithm>
#include <mutex>
#include <unordered_set>

#include "qs_host.h"

namespace {

constexpr uint32_t kEnvMagic = 0x51454e56u;  // "QENV"
constexpr uint32_t kRegMagic = 0x51524547u;  // "QREG"
constexpr uint32_t kCircMagic = 0x51435243u; // "QCRC"
constexpr uint32_t kBatchMagic = 0x51424154u; // "QBAT"

thread_local std::string g_error = "no error";

std::mutex g_handles_mu;
std::unordered_set<const void*> g_handles;

void handle_add(const void* p)
{
    std::lock_guard<std::mutex> g(g_handles_mu);
    g_handles.insert(p);
}

bool handle_remove(const void* p)
{
    std::lock_guard<std::mutex> g(g_handles_mu);
    return g_handles.erase(p) == 1;
}

bool handle_live(const void* p)
{
    std::lock_guard<std::mutex> g(g_handles_mu);
    return g_handles.count(p) == 1;
}

// QS_FAULT_ALLOC=k makes the k-th device allocation of the process fail
// (host-forced out-of-memory for the error-path tests).
std::mutex g_alloc_mu;
long g_alloc_count = 0;

hipError_t dev_alloc(void** p, size_t bytes)
{
    {
        std::lock_guard<std::mutex> g(g_alloc_mu);
        ++g_alloc_count;
        const char* f = getenv("QS_FAULT_ALLOC");
        if (f && atol(f) == g_alloc_count) return hipErrorOutOfMemory;
    }
    return hipMalloc(p, bytes);
}

// dev_alloc on a stream (stream-ordered; no device-wide synchronisation)
hipError_t dev_alloc_async(void** p, size_t bytes, hipStream_t s)
{
    {
        std::lock_guard<std::mutex> g(g_alloc_mu);
        ++g_alloc_count;
        const char* f = getenv("QS_FAULT_ALLOC");
        if (f && atol(f) == g_alloc_count) return hipErrorOutOfMemory;
    }
    return hipMallocAsync(p, bytes, s);
}

bool valid_env(qs_env e) { return e && handle_live(e) && e->magic == kEnvMagic; }
bool valid_reg(qs_reg r) { return r && handle_live(r) && r->magic == kRegMagic; }
bool valid_circ(qs_circuit c) { return c && handle_live(c) && c->magic == kCircMagic; }
bool valid_batch(qs_batch b) { return b && handle_live(b) && b->magic == kBatchMagic; }

#define QS_CHECK_REG(r) \
    if (!valid_reg(r)) return qs::set_error(QS_E_HANDLE, "invalid register handle")

#define QS_HIP(call)                                             \
    do {                                                         \
        hipError_t e_ = (call);                                  \
        if (e_ != hipSuccess) return qs::hip_error(e_, #call);   \
    } while (0)

qs::Launch launch_of(qs_reg r) { return qs::Launch{r->stream, r->env->device}; }

// Qubit list checks: each in [0, n), all distinct, none equal to `exclude`.
qs_status check_qubits(const int* qs_, int count, int n, int exclude, const char* what)
{
    if (count < 0 || count > 62) return qs::set_error(QS_E_ARG, std::string(what) + ": bad count");
    if (count > 0 && !qs_) return qs::set_error(QS_E_ARG, std::string(what) + ": NULL list");
    uint64_t seen = 0;
    for (int k = 0; k < count; ++k) {
        const int q = qs_[k];
        if (q < 0 || q >= n)
            return qs::set_error(QS_E_ARG, std::string(what) + ": qubit " + std::to_string(q) +
                                               " outside [0, " + std::to_string(n) + ")");
        if (q == exclude)
            return qs::set_error(QS_E_ARG, std::string(what) + ": control equals the target");
        if ((seen >> q) & 1) return qs::set_error(QS_E_ARG, std::string(what) + ": duplicate qubit");
        seen |= 1ull << q;
    }
    return QS_OK;
}

qs_status check_target(int t, int n)
{
    if (t < 0 || t >= n)
        return qs::set_error(QS_E_ARG, "target qubit " + std::to_string(t) + " outside [0, " +
                                           std::to_string(n) + ")");
    return QS_OK;
}

qs_status check_unitary(const qs_cplx* u)
{
    if (!u) return qs::set_error(QS_E_ARG, "NULL matrix");
    for (int k = 0; k < 4; ++k)
        if (!isfinite(u[k].re) || !isfinite(u[k].im)) return qs::set_error(QS_E_ARG, "non-finite matrix");
    // (U U^dagger)[r][c] = sum_s U[r][s] conj(U[c][s])
    double worst = 0.0;
    for (int r = 0; r < 2; ++r)
        for (int c = 0; c < 2; ++c) {
            double re = 0.0, im = 0.0;
            for (int s = 0; s < 2; ++s) {
                const qs_cplx a = u[2 * r + s], b = u[2 * c + s];
                re += a.re * b.re + a.im * b.im;
                im += a.im * b.re - a.re * b.im;
            }
            if (r == c) re -= 1.0;
            worst = std::max(worst, std::max(fabs(re), fabs(im)));
        }
    if (worst > 1e-10) return qs::set_error(QS_E_NOT_UNITARY, "matrix is not unitary");
    return QS_OK;
}

template <typename T>
qs::Mat2<T> to_mat(const double* u8)
{
    qs::Mat2<T> m;
    for (int k = 0; k < 8; ++k) m.m[k] = (T)u8[k];
    return m;
}

size_t elem_bytes(int prec) { return prec == QS_C128 ? 16 : 8; }

qs_status sync_stream(qs_reg r)
{
    QS_HIP(hipStreamSynchronize(r->stream));
    return QS_OK;
}

// --- per-operation dispatch -------------------------------------------------

template <typename T>
qs_status do_dense(qs_reg r, const int* ctrls, int nc, int t, const double* u8)
{
    const qs::Mat2<T> m = to_mat<T>(u8);
    const qs::Launch L = launch_of(r);
    if (r->kind == QS_DENSITY)
        return qs::profiled(r, QS_K_DM_GATE, [&](int*) {
            return qs::launch_dm_gate<T>(L, r->amp, r->n, t, ctrls, nc, m);
        });
    return qs::profiled(r, QS_K_GATE, [&](int* klass) {
        return qs::launch_gate<T>(L, r->amp, r->nbits, t, ctrls, nc, m, klass);
    });
}

template <typename T>
qs_status do_not(qs_reg r, const int* ctrls, int nc, int t)
{
    const qs::Launch L = launch_of(r);
    if (r->kind == QS_DENSITY) {
        const double x[8] = {0, 0, 1, 0, 1, 0, 0, 0};
        const qs::Mat2<T> m = to_mat<T>(x);
        return qs::profiled(r, QS_K_DM_GATE, [&](int*) {
            return qs::launch_dm_gate<T>(L, r->amp, r->n, t, ctrls, nc, m);
        });
    }
    return qs::profiled(r, QS_K_NOT, [&](int*) {
        return qs::launch_not<T>(L, r->amp, r->nbits, t, ctrls, nc);
    });
}

template <typename T>
qs_status do_phase(qs_reg r, const int* qubits, int nq, double angle)
{
    const qs::Launch L = launch_of(r);
    uint64_t mask = 0;
    for (int k = 0; k < nq; ++k) mask |= 1ull << qubits[k];
    const double c = cos(angle), s = sin(angle);
    if (r->kind == QS_DENSITY) {
        // rows with all bits set gain exp(i a), columns with all bits set
        // gain exp(-i a); entries with both keep their value.
        const uint64_t cmask = mask << r->n;
        qs_status st = qs::profiled(r, QS_K_PHASE, [&](int*) {
            return qs::launch_phase<T>(L, r->amp, r->nbits, mask, cmask, c, s);
        });
        if (st != QS_OK) return st;
        return qs::profiled(r, QS_K_PHASE, [&](int*) {
            return qs::launch_phase<T>(L, r->amp, r->nbits, cmask, mask, c, -s);
        });
    }
    return qs::profiled(r, QS_K_PHASE, [&](int*) {
        return qs::launch_phase<T>(L, r->amp, r->nbits, mask, 0, c, s);
    });
}

template <typename T>
qs_status do_channel(qs_reg r, int channel, int t, double p)
{
    const qs::Launch L = launch_of(r);
    return qs::profiled(r, QS_K_DM_CHANNEL, [&](int*) {
        return qs::launch_dm_channel<T>(L, r->amp, r->n, t, channel, p);
    });
}

qs_status check_channel(qs_reg r, int channel, int t, double p)
{
    if (r->kind != QS_DENSITY) return qs::set_error(QS_E_KIND, "channels need a density matrix");
    qs_status s = check_target(t, r->n);
    if (s) return s;
    double hi = 1.0;
    if (channel == QS_DEPHASING) hi = 0.5;
    else if (channel == QS_DEPOLARISING) hi = 0.75;
    else if (channel != QS_DAMPING) return qs::set_error(QS_E_ARG, "unknown channel");
    if (!(p >= 0.0 && p <= hi)) return qs::set_error(QS_E_ARG, "channel strength out of range");
    return QS_OK;
}

// Probabilities: out[0] = sum over bit q == 0, out[1] = bit q == 1 (q < 0:
// total in out[0]).  Synchronous.
// Neumaier compensated sum on the host.
struct HSum {
    double s, c;
};

void hadd(HSum& a, double v)
{
    const double t = a.s + v;
    a.c += (fabs(a.s) >= fabs(v)) ? ((a.s - t) + v) : ((v - t) + a.s);
    a.s = t;
}

qs_status probs(qs_reg r, int q, double out[2])
{
    const qs::Launch L = launch_of(r);
    double* partials = r->scratch;
    double* dev_out = r->scratch + 4 * qs::kReduceBlocks;
    qs_status st = qs::profiled(r, QS_K_REDUCE, [&](int*) {
        if (r->kind == QS_DENSITY)
            return r->prec == QS_C128 ? qs::launch_prob_dm<double>(L, r->amp, r->n, q, partials, dev_out)
                                      : qs::launch_prob_dm<float>(L, r->amp, r->n, q, partials, dev_out);
        return r->prec == QS_C128 ? qs::launch_prob_sv<double>(L, r->amp, r->nbits, q, partials, dev_out)
                                  : qs::launch_prob_sv<float>(L, r->amp, r->nbits, q, partials, dev_out);
    });
    if (st) return st;
    QS_HIP(hipMemcpyAsync(r->host_res, dev_out, 2 * sizeof(double), hipMemcpyDeviceToHost, r->stream));
    if ((st = sync_stream(r))) return st;
    out[0] = r->host_res[0];
    out[1] = r->host_res[1];
    return QS_OK;
}

}  // namespace

namespace qs {

qs_status set_error(qs_status s, const std::string& msg)
{
    g_error = msg;
    return s;
}

qs_status hip_error(hipError_t e, const char* what)
{
    g_error = std::string(what) + ": " + hipGetErrorString(e);
    return e == hipErrorOutOfMemory ? QS_E_OOM : QS_E_DEVICE;
}

qs_status apply_op(qs_reg r, const OpRec& op)
{
    const bool dbl = r->prec == QS_C128;
    const int* c = op.ctrls.data();
    const int nc = (int)op.ctrls.size();
    switch (op.kind) {
    case 0: return dbl ? do_dense<double>(r, c, nc, op.target, op.u) : do_dense<float>(r, c, nc, op.target, op.u);
    case 1: return dbl ? do_not<double>(r, c, nc, op.target) : do_not<float>(r, c, nc, op.target);
    case 2: return dbl ? do_phase<double>(r, c, nc, op.angle) : do_phase<float>(r, c, nc, op.angle);
    case 4: {  // a recorded two-qubit unitary
        qs_cplx u[16];
        for (int k = 0; k < 16; ++k) u[k] = qs_cplx{op.m4[2 * k], op.m4[2 * k + 1]};
        return qs_two_qubit_unitary(r, op.target, op.target2, u);
    }
    default:
        return dbl ? do_channel<double>(r, op.channel, op.target, op.p)
                   : do_channel<float>(r, op.channel, op.target, op.p);
    }
}

}  // namespace qs

// ===========================================================================
extern "C" {

const char* qs_last_error(void) { return g_error.c_str(); }

// ---- seeded draws: Philox4x64-10 (Salmon, Moraes, Dror, Shaw, "Parallel
// random numbers: as easy as 1, 2, 3", SC'11) -------------------------------
namespace {

struct Ctr4 {
    uint64_t v[4];
};

// The ten-round Philox bijection of a 256-bit counter under a 128-bit key:
// each round multiplies words 0 and 2 by the round constants into 128-bit
// products and mixes their halves with words 1 and 3 and the key; the key
// is bumped by the Weyl constants between rounds.
Ctr4 philox4x64_10(Ctr4 c, uint64_t k0, uint64_t k1)
{
    const uint64_t m0 = 0xD2E7470EE14C6C93ull, m1 = 0xCA5A826395121157ull;
    const uint64_t w0 = 0x9E3779B97F4A7C15ull, w1 = 0xBB67AE8584CAA73Bull;
    for (int r = 0; r < 10; ++r) {
        if (r) {
            k0 += w0;
            k1 += w1;
        }
        const unsigned __int128 p0 = (unsigned __int128)m0 * c.v[0];
        const unsigned __int128 p1 = (unsigned __int128)m1 * c.v[2];
        const uint64_t h0 = (uint64_t)(p0 >> 64), l0 = (uint64_t)p0;
        const uint64_t h1 = (uint64_t)(p1 >> 64), l1 = (uint64_t)p1;
        c = Ctr4{{h1 ^ c.v[1] ^ k0, l1, h0 ^ c.v[3] ^ k1, l0}};
    }
    return c;
}

void philox_fill(uint64_t seed, uint64_t stream, uint64_t first, int count, double* out)
{
    for (int i = 0; i < count;) {
        const uint64_t k = first + (uint64_t)i;
        // block counter k / 4 + 1 (a 256-bit integer whose upper words stay
        // 0, since k / 4 + 1 < 2^62)
        Ctr4 c = {{k / 4 + 1, 0, 0, 0}};
        c = philox4x64_10(c, seed, stream);
        for (uint64_t w = k % 4; w < 4 && i < count; ++w, ++i)
            out[i] = (double)(c.v[w] >> 11) * (1.0 / 9007199254740992.0);
    }
}

}  // namespace

qs_status qs_philox_draws(uint64_t seed, uint64_t stream, uint64_t first, int count, double* out)
{
    if (count < 0) return qs::set_error(QS_E_ARG, "negative count");
    if (count > 0 && !out) return qs::set_error(QS_E_ARG, "NULL output");
    philox_fill(seed, stream, first, count, out);
    return QS_OK;
}

qs_status qs_env_create(int device, qs_env* out)
{
    if (!out) return qs::set_error(QS_E_ARG, "NULL output");
    int count = 0;
    QS_HIP(hipGetDeviceCount(&count));
    if (device < 0 || device >= count) return qs::set_error(QS_E_ARG, "no such device");
    QS_HIP(hipSetDevice(device));
    qs_env e = new qs_env_s();
    e->magic = kEnvMagic;
    e->device = device;
    e->profile = false;
    for (int k = 0; k < QS_K_COUNT; ++k) {
        e->launches[k] = 0;
        e->ms[k] = 0.0;
    }
    handle_add(e);
    *out = e;
    return QS_OK;
}

qs_status qs_env_seed(qs_env env, uint64_t seed, uint64_t stream)
{
    if (!valid_env(env)) return qs::set_error(QS_E_HANDLE, "invalid environment handle");
    std::lock_guard<std::mutex> g(env->mu);
    env->rng_seed = seed;
    env->rng_stream = stream;
    env->rng_next = 0;
    return QS_OK;
}

qs_status qs_env_destroy(qs_env env)
{
    if (!valid_env(env) || !handle_remove(env)) return qs::set_error(QS_E_HANDLE, "invalid environment handle");
    (void)hipSetDevice(env->device);
    for (auto& rec : env->recs) {
        (void)hipEventDestroy(rec.a);
        (void)hipEventDestroy(rec.b);
    }
    for (auto& sp : env->scratch_pool) {
        (void)hipFree(sp.first);
        (void)hipHostFree(sp.second);
    }
    env->magic = 0;
    delete env;
    return QS_OK;
}

qs_status qs_env_sync(qs_env env)
{
    if (!valid_env(env)) return qs::set_error(QS_E_HANDLE, "invalid environment handle");
    QS_HIP(hipSetDevice(env->device));
    QS_HIP(hipDeviceSynchronize());
    return QS_OK;
}

qs_status qs_profile_enable(qs_env env, int enable)
{
    if (!valid_env(env)) return qs::set_error(QS_E_HANDLE, "invalid environment handle");
    env->profile = enable != 0;
    return QS_OK;
}

static qs_status fold_profile(qs_env env)
{
    QS_HIP(hipSetDevice(env->device));
    QS_HIP(hipDeviceSynchronize());
    std::lock_guard<std::mutex> g(env->mu);
    for (auto& rec : env->recs) {
        float ms = 0.0f;
        QS_HIP(hipEventElapsedTime(&ms, rec.a, rec.b));
        env->launches[rec.klass] += 1;
        env->ms[rec.klass] += ms;
        (void)hipEventDestroy(rec.a);
        (void)hipEventDestroy(rec.b);
    }
    env->recs.clear();
    return QS_OK;
}

qs_status qs_profile_read(qs_env env, int klass, uint64_t* launches, double* total_ms)
{
    if (!valid_env(env)) return qs::set_error(QS_E_HANDLE, "invalid environment handle");
    if (klass < 0 || klass >= QS_K_COUNT) return qs::set_error(QS_E_ARG, "unknown kernel class");
    qs_status s = fold_profile(env);
    if (s) return s;
    if (launches) *launches = env->launches[klass];
    if (total_ms) *total_ms = env->ms[klass];
    return QS_OK;
}

qs_status qs_profile_reset(qs_env env)
{
    if (!valid_env(env)) return qs::set_error(QS_E_HANDLE, "invalid environment handle");
    qs_status s = fold_profile(env);
    if (s) return s;
    for (int k = 0; k < QS_K_COUNT; ++k) {
        env->launches[k] = 0;
        env->ms[k] = 0.0;
    }
    return QS_OK;
}

size_t qs_reg_bytes(int n, int kind, int prec)
{
    if (prec != QS_C64 && prec != QS_C128) return 0;
    int bits;
    if (kind == QS_STATEVEC) {
        if (n < 1 || n > 40) return 0;
        bits = n;
    } else if (kind == QS_DENSITY) {
        if (n < 1 || n > 20) return 0;
        bits = 2 * n;
    } else {
        return 0;
    }
    return elem_bytes(prec) << bits;
}

static qs_status reg_common(qs_env env, int n, int kind, int prec, void* stream, qs_reg* out,
                            void* dev_ptr, size_t bytes)
{
    if (!valid_env(env)) return qs::set_error(QS_E_HANDLE, "invalid environment handle");
    if (!out) return qs::set_error(QS_E_ARG, "NULL output");
    const size_t need = qs_reg_bytes(n, kind, prec);
    if (need == 0) return qs::set_error(QS_E_ARG, "invalid qubit count, kind or precision");
    if (dev_ptr && bytes < need) return qs::set_error(QS_E_ARG, "wrapped buffer too small");
    if (dev_ptr && ((uintptr_t)dev_ptr & 15)) return qs::set_error(QS_E_ARG, "wrapped buffer not 16-byte aligned");
    QS_HIP(hipSetDevice(env->device));
    void* amp = dev_ptr;
    if (!amp) {
        const hipError_t e = dev_alloc(&amp, need);
        if (e != hipSuccess) {
            (void)hipGetLastError();
            return qs::set_error(QS_E_OOM, "cannot allocate " + std::to_string(need) + " bytes");
        }
    }
    void* scratch = nullptr;
    void* hres = nullptr;
    {
        std::lock_guard<std::mutex> g(env->mu);
        if (!env->scratch_pool.empty()) {
            scratch = env->scratch_pool.back().first;
            hres = env->scratch_pool.back().second;
            env->scratch_pool.pop_back();
        }
    }
    if (!scratch) {
        const size_t sbytes = qs::kScratchDoubles * sizeof(double);
        hipError_t e = dev_alloc(&scratch, sbytes);
        if (e == hipSuccess) e = hipHostMalloc(&hres, 2 * sizeof(double), hipHostMallocDefault);
        if (e != hipSuccess) {
            (void)hipGetLastError();
            if (scratch) (void)hipFree(scratch);
            if (!dev_ptr) (void)hipFree(amp);
            return qs::set_error(QS_E_OOM, "cannot allocate register scratch");
        }
    }
    qs_reg r = new qs_reg_s();
    r->magic = kRegMagic;
    r->env = env;
    r->n = n;
    r->nbits = kind == QS_DENSITY ? 2 * n : n;
    r->kind = kind;
    r->prec = prec;
    r->amp = amp;
    r->bytes = need;
    r->owned = dev_ptr == nullptr;
    r->stream = (hipStream_t)stream;
    r->scratch = (double*)scratch;
    r->host_res = (double*)hres;
    handle_add(r);
    *out = r;
    return QS_OK;
}

qs_status qs_reg_create(qs_env env, int n, int kind, int prec, void* hip_stream, qs_reg* out)
{
    return reg_common(env, n, kind, prec, hip_stream, out, nullptr, 0);
}

qs_status qs_reg_wrap(qs_env env, int n, int kind, int prec, void* dev_ptr, size_t bytes,
                      void* hip_stream, qs_reg* out)
{
    if (!dev_ptr) return qs::set_error(QS_E_ARG, "NULL device pointer");
    return reg_common(env, n, kind, prec, hip_stream, out, dev_ptr, bytes);
}

qs_status qs_reg_destroy(qs_reg r)
{
    if (!valid_reg(r) || !handle_remove(r)) return qs::set_error(QS_E_HANDLE, "invalid register handle");
    (void)hipSetDevice(r->env->device);
    (void)hipStreamSynchronize(r->stream);
    if (r->owned) (void)hipFree(r->amp);
    {
        std::lock_guard<std::mutex> g(r->env->mu);
        r->env->scratch_pool.push_back({r->scratch, r->host_res});
    }
    r->magic = 0;
    delete r;
    return QS_OK;
}

qs_status qs_reg_info(qs_reg r, int* n, int* kind, int* prec, void** dev_ptr, void** hip_stream)
{
    QS_CHECK_REG(r);
    if (n) *n = r->n;
    if (kind) *kind = r->kind;
    if (prec) *prec = r->prec;
    if (dev_ptr) *dev_ptr = r->amp;
    if (hip_stream) *hip_stream = (void*)r->stream;
    return QS_OK;
}

qs_status qs_init_basis(qs_reg r, uint64_t index)
{
    QS_CHECK_REG(r);
    if (r->n < 64 && index >= (1ull << r->n)) return qs::set_error(QS_E_ARG, "basis index out of range");
    const uint64_t len = 1ull << r->nbits;
    const uint64_t pos = r->kind == QS_DENSITY ? index + (index << r->n) : index;
    const qs::Launch L = launch_of(r);
    return qs::profiled(r, QS_K_INIT, [&](int*) {
        return r->prec == QS_C128 ? qs::launch_init_basis<double>(L, r->amp, len, pos, 1.0, 0.0)
                                  : qs::launch_init_basis<float>(L, r->amp, len, pos, 1.0, 0.0);
    });
}

qs_status qs_init_zero(qs_reg r) { return qs_init_basis(r, 0); }

qs_status qs_get_amps(qs_reg r, uint64_t start, uint64_t count, qs_cplx* host_out)
{
    QS_CHECK_REG(r);
    const uint64_t len = 1ull << r->nbits;
    if (start > len || count > len - start) return qs::set_error(QS_E_ARG, "amplitude range outside the register");
    if (count == 0) return QS_OK;
    if (!host_out) return qs::set_error(QS_E_ARG, "NULL host buffer");
    if (r->prec == QS_C128) {
        QS_HIP(hipMemcpyAsync(host_out, (char*)r->amp + 16 * start, 16 * count, hipMemcpyDeviceToHost, r->stream));
        return sync_stream(r);
    }
    std::vector<float> tmp(2 * count);
    QS_HIP(hipMemcpyAsync(tmp.data(), (char*)r->amp + 8 * start, 8 * count, hipMemcpyDeviceToHost, r->stream));
    qs_status s = sync_stream(r);
    if (s) return s;
    for (uint64_t i = 0; i < count; ++i) {
        host_out[i].re = tmp[2 * i];
        host_out[i].im = tmp[2 * i + 1];
    }
    return QS_OK;
}

qs_status qs_set_amps(qs_reg r, uint64_t start, uint64_t count, const qs_cplx* host_in)
{
    QS_CHECK_REG(r);
    const uint64_t len = 1ull << r->nbits;
    if (start > len || count > len - start) return qs::set_error(QS_E_ARG, "amplitude range outside the register");
    if (count == 0) return QS_OK;
    if (!host_in) return qs::set_error(QS_E_ARG, "NULL host buffer");
    if (r->prec == QS_C128) {
        QS_HIP(hipMemcpyAsync((char*)r->amp + 16 * start, host_in, 16 * count, hipMemcpyHostToDevice, r->stream));
        return sync_stream(r);
    }
    std::vector<float> tmp(2 * count);
    for (uint64_t i = 0; i < count; ++i) {
        tmp[2 * i] = (float)host_in[i].re;
        tmp[2 * i + 1] = (float)host_in[i].im;
    }
    QS_HIP(hipMemcpyAsync((char*)r->amp + 8 * start, tmp.data(), 8 * count, hipMemcpyHostToDevice, r->stream));
    return sync_stream(r);
}

qs_status qs_multi_controlled_unitary(qs_reg r, const int* controls, int n_controls, int target,
                                      const qs_cplx u[4])
{
    QS_CHECK_REG(r);
    qs_status s = check_target(target, r->n);
    if (!s) s = check_qubits(controls, n_controls, r->n, target, "controls");
    if (!s) s = check_unitary(u);
    if (s) return s;
    double u8[8];
    for (int k = 0; k < 4; ++k) {
        u8[2 * k] = u[k].re;
        u8[2 * k + 1] = u[k].im;
    }
    return r->prec == QS_C128 ? do_dense<double>(r, controls, n_controls, target, u8)
                              : do_dense<float>(r, controls, n_controls, target, u8);
}

qs_status qs_unitary(qs_reg r, int target, const qs_cplx u[4])
{
    return qs_multi_controlled_unitary(r, nullptr, 0, target, u);
}

qs_status qs_controlled_unitary(qs_reg r, int control, int target, const qs_cplx u[4])
{
    return qs_multi_controlled_unitary(r, &control, 1, target, u);
}

qs_status qs_multi_controlled_not(qs_reg r, const int* controls, int n_controls, int target)
{
    QS_CHECK_REG(r);
    qs_status s = check_target(target, r->n);
    if (!s) s = check_qubits(controls, n_controls, r->n, target, "controls");
    if (s) return s;
    return r->prec == QS_C128 ? do_not<double>(r, controls, n_controls, target)
                              : do_not<float>(r, controls, n_controls, target);
}

qs_status qs_multi_controlled_phase(qs_reg r, const int* qubits, int n_qubits, double angle)
{
    QS_CHECK_REG(r);
    if (n_qubits < 1) return qs::set_error(QS_E_ARG, "phase needs at least one qubit");
    qs_status s = check_qubits(qubits, n_qubits, r->n, -1, "qubits");
    if (s) return s;
    if (!isfinite(angle)) return qs::set_error(QS_E_ARG, "non-finite angle");
    return r->prec == QS_C128 ? do_phase<double>(r, qubits, n_qubits, angle)
                              : do_phase<float>(r, qubits, n_qubits, angle);
}

// ---- named gates ----------------------------------------------------------

qs_status qs_hadamard(qs_reg r, int target)
{
    const double s = 1.0 / sqrt(2.0);
    const qs_cplx u[4] = {{s, 0.0}, {s, 0.0}, {s, 0.0}, {-s, 0.0}};
    return qs_unitary(r, target, u);
}

qs_status qs_cnot(qs_reg r, int control, int target)
{
    return qs_multi_controlled_not(r, &control, 1, target);
}

qs_status qs_cz(qs_reg r, int q1, int q2)
{
    const int qubits[2] = {q1, q2};
    return qs_multi_controlled_phase(r, qubits, 2, M_PI);
}

qs_status qs_rotate_x(qs_reg r, int target, double theta)
{
    const double c = cos(0.5 * theta), s = sin(0.5 * theta);
    const qs_cplx u[4] = {{c, 0.0}, {0.0, -s}, {0.0, -s}, {c, 0.0}};
    return qs_unitary(r, target, u);
}

qs_status qs_rotate_y(qs_reg r, int target, double theta)
{
    const double c = cos(0.5 * theta), s = sin(0.5 * theta);
    const qs_cplx u[4] = {{c, 0.0}, {-s, 0.0}, {s, 0.0}, {c, 0.0}};
    return qs_unitary(r, target, u);
}

qs_status qs_rotate_z(qs_reg r, int target, double theta)
{
    const double c = cos(0.5 * theta), s = sin(0.5 * theta);
    const qs_cplx u[4] = {{c, -s}, {0.0, 0.0}, {0.0, 0.0}, {c, s}};
    return qs_unitary(r, target, u);
}

qs_status qs_t_gate(qs_reg r, int target)
{
    return qs_multi_controlled_phase(r, &target, 1, 0.25 * M_PI);
}

qs_status qs_sqrt_x(qs_reg r, int target)
{
    const qs_cplx u[4] = {{0.5, 0.5}, {0.5, -0.5}, {0.5, -0.5}, {0.5, 0.5}};
    return qs_unitary(r, target, u);
}

qs_status qs_sqrt_y(qs_reg r, int target)
{
    const qs_cplx u[4] = {{0.5, 0.5}, {-0.5, -0.5}, {0.5, 0.5}, {0.5, 0.5}};
    return qs_unitary(r, target, u);
}

static qs_status mix(qs_reg r, int channel, int target, double p)
{
    QS_CHECK_REG(r);
    qs_status s = check_channel(r, channel, target, p);
    if (s) return s;
    return r->prec == QS_C128 ? do_channel<double>(r, channel, target, p)
                              : do_channel<float>(r, channel, target, p);
}

qs_status qs_mix_dephasing(qs_reg r, int target, double p) { return mix(r, QS_DEPHASING, target, p); }
qs_status qs_mix_depolarising(qs_reg r, int target, double p) { return mix(r, QS_DEPOLARISING, target, p); }
qs_status qs_mix_damping(qs_reg r, int target, double gamma) { return mix(r, QS_DAMPING, target, gamma); }

qs_status qs_calc_total_prob(qs_reg r, double* out)
{
    QS_CHECK_REG(r);
    if (!out) return qs::set_error(QS_E_ARG, "NULL output");
    double v[2];
    qs_status s = probs(r, -1, v);
    if (s) return s;
    *out = v[0] + v[1];
    return QS_OK;
}

qs_status qs_calc_prob_of_outcome(qs_reg r, int qubit, int outcome, double* out)
{
    QS_CHECK_REG(r);
    if (!out) return qs::set_error(QS_E_ARG, "NULL output");
    qs_status s = check_target(qubit, r->n);
    if (s) return s;
    if (outcome != 0 && outcome != 1) return qs::set_error(QS_E_ARG, "outcome must be 0 or 1");
    // A state-vector qubit at or above the 128-byte line (8 complex128 or 16
    // complex64 amplitudes) splits the state into halves of whole lines:
    // read only the outcome's half.
    if (r->kind == QS_STATEVEC && qubit >= (r->prec == QS_C128 ? 3 : 4)) {
        const qs::Launch L = launch_of(r);
        double* partials = r->scratch;
        double* dev_out = r->scratch + 4 * qs::kReduceBlocks;
        s = qs::profiled(r, QS_K_REDUCE, [&](int*) {
            return r->prec == QS_C128
                       ? qs::launch_prob_half_sv<double>(L, r->amp, r->nbits, qubit, outcome, partials, dev_out)
                       : qs::launch_prob_half_sv<float>(L, r->amp, r->nbits, qubit, outcome, partials, dev_out);
        });
        if (s) return s;
        QS_HIP(hipMemcpyAsync(r->host_res, dev_out, 2 * sizeof(double), hipMemcpyDeviceToHost, r->stream));
        if ((s = sync_stream(r))) return s;
        *out = r->host_res[0];
        return QS_OK;
    }
    double v[2];
    if ((s = probs(r, qubit, v))) return s;
    *out = v[outcome];
    return QS_OK;
}

// The outcome from the draw and the probabilities v = {P(0), P(1)}, then
// the collapse onto it.
static qs_status measure_with(qs_reg r, int qubit, const double v[2], double u01, int* outcome, double* prob)
{
    qs_status s = QS_OK;
    double p0 = v[0];
    if (p0 < 0.0) p0 = 0.0;
    if (p0 > 1.0) p0 = 1.0;
    const int o = (u01 < p0) ? 0 : 1;
    const double p = v[o];
    if (!(p > 0.0)) return qs::set_error(QS_E_ARG, "selected outcome has zero probability");
    const qs::Launch L = launch_of(r);
    if (r->kind == QS_DENSITY) {
        const double scale = 1.0 / p;
        s = qs::profiled(r, QS_K_COLLAPSE, [&](int*) {
            return r->prec == QS_C128 ? qs::launch_collapse_dm<double>(L, r->amp, r->n, qubit, o, scale)
                                      : qs::launch_collapse_dm<float>(L, r->amp, r->n, qubit, o, scale);
        });
    } else {
        const double scale = 1.0 / sqrt(p);
        s = qs::profiled(r, QS_K_COLLAPSE, [&](int*) {
            return r->prec == QS_C128 ? qs::launch_collapse_sv<double>(L, r->amp, r->nbits, qubit, o, scale)
                                      : qs::launch_collapse_sv<float>(L, r->amp, r->nbits, qubit, o, scale);
        });
    }
    if (s) return s;
    if (outcome) *outcome = o;
    if (prob) *prob = p;
    return QS_OK;
}

qs_status qs_measure(qs_reg r, int qubit, double u01, int* outcome, double* prob)
{
    QS_CHECK_REG(r);
    qs_status s = check_target(qubit, r->n);
    if (s) return s;
    if (!(u01 >= 0.0 && u01 < 1.0)) return qs::set_error(QS_E_ARG, "draw must lie in [0, 1)");
    double v[2];
    if ((s = probs(r, qubit, v))) return s;
    return measure_with(r, qubit, v, u01, outcome, prob);
}

qs_status qs_measure_given_probs(qs_reg r, int qubit, double p0, double p1, double u01, int* outcome, double* prob)
{
    QS_CHECK_REG(r);
    qs_status s = check_target(qubit, r->n);
    if (s) return s;
    if (!(u01 >= 0.0 && u01 < 1.0)) return qs::set_error(QS_E_ARG, "draw must lie in [0, 1)");
    if (!(p0 >= 0.0 && p1 >= 0.0 && std::isfinite(p0) && std::isfinite(p1)))
        return qs::set_error(QS_E_ARG, "outcome probabilities must be finite and non-negative");
    const double v[2] = {p0, p1};
    return measure_with(r, qubit, v, u01, outcome, prob);
}

// Measure qubits 0..n-1 in turn.  Step k's numbers are those qs_measure
// would compute on the state left by steps 0..k-1: with W(S) the sum of
// |alpha|^2 (state vector) or of diagonal entries (density matrix) of the
// ORIGINAL state over the set S of indices that agree with the outcomes so
// far, and g = product of 1/p over those steps, p0 = W(S, bit k = 0) * g
// clamped to [0, 1], outcome = (u < p0) ? 0 : 1, p = W(S, bit k = outcome) * g.
// The W sums come from compensated histograms over 10 qubits at a time (the
// first over the whole state, each later one over the surviving subspace),
// and the state is collapsed once at the end: the measured basis entry
// times sqrt(g) (state vector) or g (density matrix), every other entry 0.
qs_status qs_measure_all(qs_reg r, const double* u01, int* outcomes, double* probs)
{
    QS_CHECK_REG(r);
    if (!u01) return qs::set_error(QS_E_ARG, "NULL draws");
    const int n = r->n;
    for (int k = 0; k < n; ++k)
        if (!(u01[k] >= 0.0 && u01[k] < 1.0)) return qs::set_error(QS_E_ARG, "draw must lie in [0, 1)");
    const qs::Launch L = launch_of(r);
    const bool dbl = r->prec == QS_C128;
    std::vector<int> out_o(n);
    std::vector<double> out_p(n);
    double g = 1.0;
    uint64_t pattern = 0;
    // one step of the walk over bins: w[b] = (sum, compensation) of W over
    // the bins of the current group; bits below k of b must match `sub`
    auto walk = [&](const std::vector<double>& w, int nbins_log, int first_qubit) -> qs_status {
        for (int k = 0; k < nbins_log; ++k) {
            const uint64_t sub = (pattern >> first_qubit) & ((1ull << k) - 1);
            HSum w0 = {0.0, 0.0}, w1 = {0.0, 0.0};
            for (uint64_t b = 0; b < (1ull << nbins_log); ++b) {
                if ((b & ((1ull << k) - 1)) != sub) continue;
                HSum& acc = ((b >> k) & 1) ? w1 : w0;
                hadd(acc, w[2 * b]);
                hadd(acc, w[2 * b + 1]);
            }
            double p0 = (w0.s + w0.c) * g;
            if (p0 < 0.0) p0 = 0.0;
            if (p0 > 1.0) p0 = 1.0;
            const int q = first_qubit + k;
            const int o = (u01[q] < p0) ? 0 : 1;
            const double p = ((o ? w1.s + w1.c : w0.s + w0.c)) * g;
            if (!(p > 0.0)) return qs::set_error(QS_E_ARG, "selected outcome has zero probability");
            out_o[q] = o;
            out_p[q] = p;
            g /= p;
            pattern |= (uint64_t)o << q;
        }
        return QS_OK;
    };
    qs_status s = QS_OK;
    if (r->kind == QS_DENSITY) {
        const uint64_t dim = 1ull << n;
        double* dd = nullptr;
        QS_HIP(hipMallocAsync((void**)&dd, dim * sizeof(double), r->stream));
        s = qs::profiled(r, QS_K_REDUCE, [&](int*) {
            return dbl ? qs::launch_diag_dm<double>(L, r->amp, n, dd) : qs::launch_diag_dm<float>(L, r->amp, n, dd);
        });
        std::vector<double> diag(dim);
        if (!s) {
            hipError_t e = hipMemcpyAsync(diag.data(), dd, dim * sizeof(double), hipMemcpyDeviceToHost, r->stream);
            if (e == hipSuccess) e = hipStreamSynchronize(r->stream);
            if (e != hipSuccess) s = qs::hip_error(e, "diagonal copy");
        }
        (void)hipFreeAsync(dd, r->stream);
        if (s) return s;
        std::vector<double> w(2 * dim, 0.0);  // (value, 0) pairs: the walk over all N qubits at once
        for (uint64_t j = 0; j < dim; ++j) w[2 * j] = diag[j];
        if ((s = walk(w, n, 0))) return s;
    } else {
        const int kb = qs::kHistBlocks;
        double* buf = nullptr;
        QS_HIP(hipMallocAsync((void**)&buf, (2 * 1024 * (size_t)kb + 2 * 1024) * sizeof(double), r->stream));
        double* dev_out = buf + 2 * 1024 * (size_t)kb;
        std::vector<double> w;
        for (int shift = 0; shift < n && !s; shift += 10) {
            const int mb = std::min(10, n - shift);
            s = qs::profiled(r, QS_K_REDUCE, [&](int*) {
                return dbl ? qs::launch_hist_sv<double>(L, r->amp, r->nbits, shift, pattern, mb, buf, kb, dev_out)
                           : qs::launch_hist_sv<float>(L, r->amp, r->nbits, shift, pattern, mb, buf, kb, dev_out);
            });
            if (s) break;
            w.assign(2ull << mb, 0.0);
            hipError_t e = hipMemcpyAsync(w.data(), dev_out, w.size() * sizeof(double), hipMemcpyDeviceToHost,
                                          r->stream);
            if (e == hipSuccess) e = hipStreamSynchronize(r->stream);
            if (e != hipSuccess) s = qs::hip_error(e, "histogram copy");
            if (!s) s = walk(w, mb, shift);
        }
        (void)hipFreeAsync(buf, r->stream);
        if (s) return s;
    }
    // the kept entry, scaled in double precision
    const uint64_t pos = r->kind == QS_DENSITY ? pattern + (pattern << n) : pattern;
    double re = 0.0, im = 0.0;
    if (dbl) {
        double v[2];
        QS_HIP(hipMemcpyAsync(v, (const double*)r->amp + 2 * pos, sizeof(v), hipMemcpyDeviceToHost, r->stream));
        if ((s = sync_stream(r))) return s;
        re = v[0];
        im = v[1];
    } else {
        float v[2];
        QS_HIP(hipMemcpyAsync(v, (const float*)r->amp + 2 * pos, sizeof(v), hipMemcpyDeviceToHost, r->stream));
        if ((s = sync_stream(r))) return s;
        re = v[0];
        im = v[1];
    }
    const double scale = r->kind == QS_DENSITY ? g : sqrt(g);
    s = qs::profiled(r, QS_K_COLLAPSE, [&](int*) {
        const uint64_t len = 1ull << r->nbits;
        return dbl ? qs::launch_init_basis<double>(L, r->amp, len, pos, re * scale, im * scale)
                   : qs::launch_init_basis<float>(L, r->amp, len, pos, re * scale, im * scale);
    });
    if (s) return s;
    for (int k = 0; k < n; ++k) {
        if (outcomes) outcomes[k] = out_o[k];
        if (probs) probs[k] = out_p[k];
    }
    return QS_OK;
}

// Draws [first, first + count) of the register's environment stream, and
// the first index; the stream is advanced by the caller on success.
namespace {
uint64_t next_draws(qs_reg r, int count, double* out)
{
    std::lock_guard<std::mutex> g(r->env->mu);
    philox_fill(r->env->rng_seed, r->env->rng_stream, r->env->rng_next, count, out);
    return r->env->rng_next;
}

void advance_draws(qs_reg r, uint64_t first, int count)
{
    std::lock_guard<std::mutex> g(r->env->mu);
    // another call may have advanced the stream meanwhile: move on from
    // whichever is further
    r->env->rng_next = std::max(r->env->rng_next, first + (uint64_t)count);
}
}  // namespace

qs_status qs_measure_seeded(qs_reg r, int qubit, int* outcome, double* prob)
{
    QS_CHECK_REG(r);
    double u = 0.0;
    const uint64_t first = next_draws(r, 1, &u);
    const qs_status s = qs_measure(r, qubit, u, outcome, prob);
    if (s == QS_OK) advance_draws(r, first, 1);
    return s;
}

qs_status qs_measure_all_seeded(qs_reg r, int* outcomes, double* probs)
{
    QS_CHECK_REG(r);
    std::vector<double> u(r->n);
    const uint64_t first = next_draws(r, r->n, u.data());
    const qs_status s = qs_measure_all(r, u.data(), outcomes, probs);
    if (s == QS_OK) advance_draws(r, first, r->n);
    return s;
}

// --- circuits ----------------------------------------------------------------

qs_status qs_circuit_create(qs_circuit* out)
{
    if (!out) return qs::set_error(QS_E_ARG, "NULL output");
    qs_circuit c = new qs_circuit_s();
    c->magic = kCircMagic;
    handle_add(c);
    *out = c;
    return QS_OK;
}

qs_status qs_circuit_destroy(qs_circuit c)
{
    if (!valid_circ(c) || !handle_remove(c)) return qs::set_error(QS_E_HANDLE, "invalid circuit handle");
    c->magic = 0;
    qs::jit_plan_free(c->jit);
    delete c;
    return QS_OK;
}

qs_status qs_circuit_size(qs_circuit c, int* n_ops)
{
    if (!valid_circ(c)) return qs::set_error(QS_E_HANDLE, "invalid circuit handle");
    if (!n_ops) return qs::set_error(QS_E_ARG, "NULL output");
    *n_ops = (int)c->ops.size();
    return QS_OK;
}

// Qubit ranges are checked again against the register at run time.
static qs_status circ_common(qs_circuit c, const int* qs_, int nq, int target, OpRec& op)
{
    if (!valid_circ(c)) return qs::set_error(QS_E_HANDLE, "invalid circuit handle");
    qs_status s = check_qubits(qs_, nq, 64, target, "qubits");
    if (s) return s;
    op.ctrls.assign(qs_, qs_ + nq);
    op.target = target;
    return QS_OK;
}

qs_status qs_circuit_add_unitary(qs_circuit c, const int* controls, int n_controls, int target,
                                 const qs_cplx u[4])
{
    OpRec op{};
    qs_status s = circ_common(c, controls, n_controls, target, op);
    if (!s && target < 0) s = qs::set_error(QS_E_ARG, "negative target");
    if (!s) s = check_unitary(u);
    if (s) return s;
    op.kind = 0;
    for (int k = 0; k < 4; ++k) {
        op.u[2 * k] = u[k].re;
        op.u[2 * k + 1] = u[k].im;
    }
    c->ops.push_back(op);
    return QS_OK;
}

qs_status qs_circuit_set_unitary(qs_circuit c, int index, const qs_cplx u[4])
{
    if (!valid_circ(c)) return qs::set_error(QS_E_HANDLE, "invalid circuit handle");
    if (index < 0 || index >= (int)c->ops.size() || c->ops[index].kind != 0)
        return qs::set_error(QS_E_ARG, "no unitary at that index");
    qs_status s = check_unitary(u);
    if (s) return s;
    for (int k = 0; k < 4; ++k) {
        c->ops[index].u[2 * k] = u[k].re;
        c->ops[index].u[2 * k + 1] = u[k].im;
    }
    ++c->version;
    return QS_OK;
}

qs_status qs_circuit_set_phase(qs_circuit c, int index, double angle)
{
    if (!valid_circ(c)) return qs::set_error(QS_E_HANDLE, "invalid circuit handle");
    if (index < 0 || index >= (int)c->ops.size() || c->ops[index].kind != 2)
        return qs::set_error(QS_E_ARG, "no phase at that index");
    if (!isfinite(angle)) return qs::set_error(QS_E_ARG, "non-finite angle");
    c->ops[index].angle = angle;
    ++c->version;
    return QS_OK;
}

qs_status qs_circuit_add_not(qs_circuit c, const int* controls, int n_controls, int target)
{
    OpRec op{};
    qs_status s = circ_common(c, controls, n_controls, target, op);
    if (!s && target < 0) s = qs::set_error(QS_E_ARG, "negative target");
    if (s) return s;
    op.kind = 1;
    c->ops.push_back(op);
    return QS_OK;
}

qs_status qs_circuit_add_phase(qs_circuit c, const int* qubits, int n_qubits, double angle)
{
    OpRec op{};
    if (n_qubits < 1) return qs::set_error(QS_E_ARG, "phase needs at least one qubit");
    qs_status s = circ_common(c, qubits, n_qubits, -1, op);
    if (!s && !isfinite(angle)) s = qs::set_error(QS_E_ARG, "non-finite angle");
    if (s) return s;
    op.kind = 2;
    op.angle = angle;
    c->ops.push_back(op);
    return QS_OK;
}

qs_status qs_circuit_add_channel(qs_circuit c, int channel, int target, double p)
{
    if (!valid_circ(c)) return qs::set_error(QS_E_HANDLE, "invalid circuit handle");
    double hi = channel == QS_DEPHASING ? 0.5 : channel == QS_DEPOLARISING ? 0.75 : 1.0;
    if (channel < QS_DEPHASING || channel > QS_DAMPING) return qs::set_error(QS_E_ARG, "unknown channel");
    if (target < 0) return qs::set_error(QS_E_ARG, "negative target");
    if (!(p >= 0.0 && p <= hi)) return qs::set_error(QS_E_ARG, "channel strength out of range");
    OpRec op{};
    op.kind = 3;
    op.channel = channel;
    op.target = target;
    op.p = p;
    c->ops.push_back(op);
    return QS_OK;
}

static qs_status circuit_check(qs_reg r, qs_circuit c)
{
    QS_CHECK_REG(r);
    if (!valid_circ(c)) return qs::set_error(QS_E_HANDLE, "invalid circuit handle");
    // Validate every op against this register before launching anything.
    for (const OpRec& op : c->ops) {
        if (op.kind == 3) {
            qs_status s = check_channel(r, op.channel, op.target, op.p);
            if (s) return s;
            continue;
        }
        if (op.kind != 2) {
            qs_status s = check_target(op.target, r->n);
            if (!s && op.kind == 4) s = check_target(op.target2, r->n);
            if (s) return s;
        }
        for (int q : op.ctrls)
            if (q >= r->n) return qs::set_error(QS_E_ARG, "circuit qubit outside the register");
    }
    return QS_OK;
}

static qs_status circuit_unfused(qs_reg r, qs_circuit c, int* n_passes)
{
    for (const OpRec& op : c->ops) {
        qs_status s = qs::apply_op(r, op);
        if (s) return s;
    }
    if (n_passes) *n_passes = (int)c->ops.size();
    return QS_OK;
}

qs_status qs_circuit_run(qs_reg r, qs_circuit c, int fusion_qubits, int* n_passes)
{
    qs_status s = circuit_check(r, c);
    if (s) return s;
    if (fusion_qubits < 0) return qs::set_error(QS_E_ARG, "negative fusion width");
    if (fusion_qubits > 0 && r->kind == QS_STATEVEC)
        return qs::run_fused_sv(r, c->ops, qs::default_fused_config(r->prec, fusion_qubits, r->n), n_passes);
    if (fusion_qubits > 0 && r->kind == QS_DENSITY) {
        // density matrices fuse through the compiled passes on their 2N-qubit vector
        qs::FusedConfig cfg = qs::default_fused_config(r->prec, fusion_qubits, r->nbits);
        if (cfg.TB != 0) {
            cfg.contig = std::min(4, cfg.TB);
            return qs::run_compiled_sv(r, c, cfg, n_passes);
        }
    }
    return circuit_unfused(r, c, n_passes);
}

qs_status qs_circuit_run_tiled(qs_reg r, qs_circuit c, int tile_qubits, int thread_bits, int max_phases,
                               int* n_passes)
{
    qs_status s = circuit_check(r, c);
    if (s) return s;
    const int RB = tile_qubits - thread_bits;
    if (!qs::fused_shape_supported(r->prec, thread_bits, RB))
        return qs::set_error(QS_E_ARG, "unsupported tile shape");
    if (tile_qubits > r->nbits) return qs::set_error(QS_E_ARG, "tile wider than the register");
    if (max_phases < 0) return qs::set_error(QS_E_ARG, "negative phase cap");
    return qs::run_fused_sv(r, c->ops, qs::FusedConfig{thread_bits, RB, max_phases}, n_passes);
}

// Shapes the run-time compiled passes accept: 6..10 thread bits, 1..5
// register bits, the tile in at most 160 KiB of LDS.
static qs_status check_compiled_shape(int prec, int n, int tile_qubits, int thread_bits, int max_phases,
                                      int contig)
{
    if (contig < 0 || contig > 6 || contig > thread_bits) return qs::set_error(QS_E_ARG, "bad contiguous-qubit count");
    const int RB = tile_qubits - thread_bits;
    if (thread_bits < 6 || thread_bits > 10 || RB < 1 || RB > 5)
        return qs::set_error(QS_E_ARG, "unsupported tile shape");
    if ((elem_bytes(prec) << tile_qubits) > 160u * 1024u) return qs::set_error(QS_E_ARG, "tile exceeds LDS");
    if (tile_qubits > n) return qs::set_error(QS_E_ARG, "tile wider than the register");
    if (max_phases < 0) return qs::set_error(QS_E_ARG, "negative phase cap");
    return QS_OK;
}

qs_status qs_circuit_run_compiled(qs_reg r, qs_circuit c, int tile_qubits, int thread_bits, int max_phases,
                                  int contig_qubits, int* n_passes)
{
    qs_status s = circuit_check(r, c);
    if (s) return s;
    if ((s = check_compiled_shape(r->prec, r->nbits, tile_qubits, thread_bits, max_phases, contig_qubits))) return s;
    qs::FusedConfig cfg{thread_bits, tile_qubits - thread_bits, max_phases};
    cfg.contig = contig_qubits ? contig_qubits : std::min(6, r->nbits);
    return qs::run_compiled_sv(r, c, cfg, n_passes);
}

qs_status qs_circuit_run_compiled_probs(qs_reg r, qs_circuit c, int tile_qubits, int thread_bits, int max_phases,
                                        int contig_qubits, const uint64_t* basis_index, double* probs_out,
                                        int* n_passes)
{
    qs_status s = circuit_check(r, c);
    if (s) return s;
    if (r->kind != QS_STATEVEC) return qs::set_error(QS_E_KIND, "readouts of compiled passes need a state vector");
    if (!probs_out) return qs::set_error(QS_E_ARG, "NULL output");
    if ((s = check_compiled_shape(r->prec, r->nbits, tile_qubits, thread_bits, max_phases, contig_qubits))) return s;
    if (basis_index && r->n < 64 && *basis_index >= (1ull << r->n))
        return qs::set_error(QS_E_ARG, "basis index out of range");
    qs::FusedConfig cfg{thread_bits, tile_qubits - thread_bits, max_phases};
    cfg.contig = contig_qubits ? contig_qubits : std::min(6, r->nbits);
    return qs::run_compiled_sv(r, c, cfg, n_passes, basis_index, probs_out);
}

qs_status qs_circuit_run_compiled_from_basis(qs_reg r, qs_circuit c, int tile_qubits, int thread_bits,
                                             int max_phases, int contig_qubits, uint64_t basis_index,
                                             int* n_passes)
{
    qs_status s = circuit_check(r, c);
    if (s) return s;
    if ((s = check_compiled_shape(r->prec, r->nbits, tile_qubits, thread_bits, max_phases, contig_qubits))) return s;
    if (r->n < 64 && basis_index >= (1ull << r->n)) return qs::set_error(QS_E_ARG, "basis index out of range");
    qs::FusedConfig cfg{thread_bits, tile_qubits - thread_bits, max_phases};
    cfg.contig = contig_qubits ? contig_qubits : std::min(6, r->nbits);
    return qs::run_compiled_sv(r, c, cfg, n_passes, &basis_index);
}

namespace {

// The generated pass set of `c` for an n-qubit register (sources and kernel data).
qs_status generated_passes(qs_circuit c, int n, int kind, int prec, int tile_qubits, int thread_bits,
                           int max_phases, int contig_qubits, std::vector<std::string>& srcs,
                           std::vector<std::vector<double>>& mats, bool readout = false)
{
    if (!valid_circ(c)) return qs::set_error(QS_E_HANDLE, "invalid circuit handle");
    if (prec != QS_C64 && prec != QS_C128) return qs::set_error(QS_E_ARG, "unknown precision");
    if (qs_reg_bytes(n, kind, prec) == 0) return qs::set_error(QS_E_ARG, "invalid qubit count or kind");
    const int nbits = kind == QS_DENSITY ? 2 * n : n;
    qs_status s = check_compiled_shape(prec, nbits, tile_qubits, thread_bits, max_phases, contig_qubits);
    if (s) return s;
    for (const OpRec& op : c->ops) {
        if (op.kind == 3 && kind != QS_DENSITY) return qs::set_error(QS_E_KIND, "channels need a density matrix");
        if (op.kind != 2 && op.target >= n) return qs::set_error(QS_E_ARG, "circuit qubit outside the register");
        if (op.kind == 4 && op.target2 >= n) return qs::set_error(QS_E_ARG, "circuit qubit outside the register");
        for (int q : op.ctrls)
            if (q >= n) return qs::set_error(QS_E_ARG, "circuit qubit outside the register");
    }
    qs::FusedConfig cfg{thread_bits, tile_qubits - thread_bits, max_phases};
    cfg.contig = contig_qubits ? contig_qubits : std::min(6, nbits);
    return qs::generate_sources(c->ops, n, kind, prec, cfg, srcs, &mats, readout);
}

}  // namespace

qs_status qs_circuit_source(qs_circuit c, int n, int kind, int prec, int tile_qubits, int thread_bits,
                            int max_phases, int contig_qubits, int pass, char* buf, size_t cap, size_t* len,
                            int* n_passes)
{
    std::vector<std::string> srcs;
    std::vector<std::vector<double>> mats;
    qs_status s = generated_passes(c, n, kind, prec, tile_qubits, thread_bits, max_phases, contig_qubits, srcs, mats,
                                   pass == -1);
    if (s) return s;
    if (n_passes) *n_passes = (int)srcs.size();
    if (pass == -1) pass = (int)srcs.size() - 1;
    if (pass < 0 || pass >= (int)srcs.size()) return qs::set_error(QS_E_ARG, "no such pass");
    const std::string& src = srcs[pass];
    if (len) *len = src.size();
    if (buf && cap > 0) {
        const size_t k = std::min(cap - 1, src.size());
        memcpy(buf, src.data(), k);
        buf[k] = '\0';
    }
    return QS_OK;
}

qs_status qs_circuit_pass_data(qs_circuit c, int n, int kind, int prec, int tile_qubits, int thread_bits,
                               int max_phases, int contig_qubits, int pass, double* buf, size_t cap, size_t* len,
                               int* n_passes)
{
    std::vector<std::string> srcs;
    std::vector<std::vector<double>> mats;
    qs_status s = generated_passes(c, n, kind, prec, tile_qubits, thread_bits, max_phases, contig_qubits, srcs, mats);
    if (s) return s;
    if (n_passes) *n_passes = (int)srcs.size();
    if (pass < 0 || pass >= (int)srcs.size()) return qs::set_error(QS_E_ARG, "no such pass");
    const std::vector<double>& m = mats[pass];
    if (len) *len = m.size();
    if (cap > 0 && !buf) return qs::set_error(QS_E_ARG, "null buffer");
    if (cap > 0) memcpy(buf, m.data(), std::min(cap, m.size()) * sizeof(double));
    return QS_OK;
}


// --- batches -----------------------------------------------------------------

static void batch_free(qs_batch b)
{
    if (b->stream) (void)hipStreamSynchronize(b->stream);  // uploads read host buffers freed below
    qs::batch_plans_free(b->plans);
    if (b->exec) (void)hipGraphExecDestroy(b->exec);
    if (b->graph) (void)hipGraphDestroy(b->graph);
    // stream-ordered frees (the batch's own work is complete: callers
    // synchronise its stream first)
    if (b->dbuf) (void)(b->stream ? hipFreeAsync(b->dbuf, b->stream) : hipFree(b->dbuf));
    if (b->dprobs) (void)(b->stream ? hipFreeAsync(b->dprobs, b->stream) : hipFree(b->dprobs));
    if (b->hprobs) (void)hipHostFree(b->hprobs);
    if (b->ev_in) (void)hipEventDestroy(b->ev_in);
    if (b->ev_out) (void)hipEventDestroy(b->ev_out);
    if (b->stream) (void)hipStreamDestroy(b->stream);
    b->magic = 0;
    delete b;
}

qs_status qs_batch_create(const qs_reg* regs, const qs_circuit* circuits, int count, int tile_qubits,
                          qs_batch* out)
{
    if (!out || !regs || !circuits || count < 1) return qs::set_error(QS_E_ARG, "empty batch");
    std::vector<qs_reg> rv;
    std::vector<const std::vector<OpRec>*> cv;
    for (int i = 0; i < count; ++i) {
        qs_status s = circuit_check(regs[i], circuits[i]);
        if (s) return s;
        const qs_reg r = regs[i];
        if (r->kind != QS_STATEVEC) return qs::set_error(QS_E_KIND, "batches hold state vectors");
        if (r->env != regs[0]->env || r->prec != regs[0]->prec)
            return qs::set_error(QS_E_ARG, "batched registers must share environment and precision");
        for (const OpRec& op : circuits[i]->ops)
            if (op.kind == 3) return qs::set_error(QS_E_KIND, "channels need a density matrix");
        rv.push_back(r);
        cv.push_back(&circuits[i]->ops);
    }
    if (tile_qubits < 9) return qs::set_error(QS_E_ARG, "tile must hold at least 9 qubits");
    QS_HIP(hipSetDevice(regs[0]->env->device));
    qs_batch b = new qs_batch_s();
    b->magic = kBatchMagic;
    b->env = regs[0]->env;
    b->prec = regs[0]->prec;
    b->count = count;
    b->regs = rv;
    b->stream = nullptr;
    b->ev_in = b->ev_out = nullptr;
    for (qs_reg r : rv)
        if (std::find(b->reg_streams.begin(), b->reg_streams.end(), r->stream) == b->reg_streams.end())
            b->reg_streams.push_back(r->stream);
    hipError_t e = hipStreamCreateWithFlags(&b->stream, hipStreamNonBlocking);
    if (e == hipSuccess) e = hipEventCreateWithFlags(&b->ev_in, hipEventDisableTiming);
    if (e == hipSuccess) e = hipEventCreateWithFlags(&b->ev_out, hipEventDisableTiming);
    if (e == hipSuccess) e = dev_alloc_async((void**)&b->dprobs, 2 * sizeof(double) * count, b->stream);
    if (e != hipSuccess) {
        (void)hipGetLastError();
        batch_free(b);
        return qs::hip_error(e, "batch resources");
    }
    qs_status s = qs::batch_build(b, rv, cv, tile_qubits);
    if (s) {
        batch_free(b);
        return s;
    }
    handle_add(b);
    *out = b;
    return QS_OK;
}

qs_status qs_batch_destroy(qs_batch b)
{
    if (!valid_batch(b) || !handle_remove(b)) return qs::set_error(QS_E_HANDLE, "invalid batch handle");
    (void)hipSetDevice(b->env->device);
    (void)hipStreamSynchronize(b->stream);
    batch_free(b);
    return QS_OK;
}

// The batch stream waits for the registers' streams; afterwards they wait for it.
static qs_status batch_enter(qs_batch b)
{
    for (hipStream_t s : b->reg_streams) {
        QS_HIP(hipEventRecord(b->ev_in, s));
        QS_HIP(hipStreamWaitEvent(b->stream, b->ev_in, 0));
    }
    return QS_OK;
}

static qs_status batch_leave(qs_batch b)
{
    QS_HIP(hipEventRecord(b->ev_out, b->stream));
    for (hipStream_t s : b->reg_streams) QS_HIP(hipStreamWaitEvent(s, b->ev_out, 0));
    return QS_OK;
}

static qs_status batch_profiled(qs_batch b, hipError_t (*fn)(qs_batch, int), int arg)
{
    qs_env env = b->env;
    hipEvent_t a = nullptr, c = nullptr;
    if (env->profile) {
        QS_HIP(hipEventCreate(&a));
        QS_HIP(hipEventCreate(&c));
        QS_HIP(hipEventRecord(a, b->stream));
    }
    const hipError_t e = fn(b, arg);
    if (env->profile) {
        QS_HIP(hipEventRecord(c, b->stream));
        std::lock_guard<std::mutex> g(env->mu);
        env->recs.push_back({QS_K_FUSED, a, c});
    }
    if (e != hipSuccess) return qs::hip_error(e, "batch launch");
    return QS_OK;
}

qs_status qs_batch_run(qs_batch b, int init_zero)
{
    if (!valid_batch(b)) return qs::set_error(QS_E_HANDLE, "invalid batch handle");
    QS_HIP(hipSetDevice(b->env->device));
    qs_status s = batch_enter(b);
    if (s) return s;
    s = batch_profiled(b, [](qs_batch bb, int init) { return qs::batch_launch(bb, init); }, init_zero ? 1 : 0);
    if (s) return s;
    return batch_leave(b);
}

qs_status qs_batch_capture(qs_batch b, int init_zero)
{
    if (!valid_batch(b)) return qs::set_error(QS_E_HANDLE, "invalid batch handle");
    QS_HIP(hipSetDevice(b->env->device));
    QS_HIP(hipStreamSynchronize(b->stream));
    if (b->exec) {
        (void)hipGraphExecDestroy(b->exec);
        b->exec = nullptr;
    }
    if (b->graph) {
        (void)hipGraphDestroy(b->graph);
        b->graph = nullptr;
    }
    QS_HIP(hipStreamBeginCapture(b->stream, hipStreamCaptureModeThreadLocal));
    const hipError_t le = qs::batch_launch(b, init_zero ? 1 : 0);
    hipGraph_t g = nullptr;
    const hipError_t ce = hipStreamEndCapture(b->stream, &g);
    if (le != hipSuccess) {
        if (g) (void)hipGraphDestroy(g);
        return qs::hip_error(le, "batch launch under capture");
    }
    if (ce != hipSuccess) return qs::hip_error(ce, "hipStreamEndCapture");
    b->graph = g;
    QS_HIP(hipGraphInstantiate(&b->exec, b->graph, nullptr, nullptr, 0));
    return QS_OK;
}

qs_status qs_batch_replay(qs_batch b)
{
    if (!valid_batch(b)) return qs::set_error(QS_E_HANDLE, "invalid batch handle");
    if (!b->exec) return qs::set_error(QS_E_ARG, "nothing captured");
    QS_HIP(hipSetDevice(b->env->device));
    qs_status s = batch_enter(b);
    if (s) return s;
    s = batch_profiled(b, [](qs_batch bb, int) { return hipGraphLaunch(bb->exec, bb->stream); }, 0);
    if (s) return s;
    return batch_leave(b);
}

qs_status qs_batch_update(qs_batch b)
{
    if (!valid_batch(b)) return qs::set_error(QS_E_HANDLE, "invalid batch handle");
    QS_HIP(hipSetDevice(b->env->device));
    return qs::batch_update(b);
}

qs_status qs_batch_probs(qs_batch b, int qubit, double* p0, double* total)
{
    if (!valid_batch(b)) return qs::set_error(QS_E_HANDLE, "invalid batch handle");
    for (qs_reg r : b->regs)
        if (qubit < 0 || qubit >= r->n) return qs::set_error(QS_E_ARG, "qubit outside a batched register");
    QS_HIP(hipSetDevice(b->env->device));
    qs_status s = batch_enter(b);
    if (s) return s;
    s = batch_profiled(b, [](qs_batch bb, int q) { return qs::batch_probs_launch(bb, q, bb->dprobs); }, qubit);
    if (s) return s;
    if (!b->hprobs)  // pinned, on first use (batches that never read probabilities need none)
        QS_HIP(hipHostMalloc((void**)&b->hprobs, 2 * sizeof(double) * b->count, hipHostMallocDefault));
    QS_HIP(hipMemcpyAsync(b->hprobs, b->dprobs, 2 * sizeof(double) * b->count, hipMemcpyDeviceToHost, b->stream));
    QS_HIP(hipStreamSynchronize(b->stream));
    for (int i = 0; i < b->count; ++i) {
        if (p0) p0[i] = b->hprobs[2 * i];
        if (total) total[i] = b->hprobs[2 * i + 1];
    }
    return batch_leave(b);
}

qs_status qs_batch_info(qs_batch b, int* n_regs, int* tile_qubits, int* n_passes)
{
    if (!valid_batch(b)) return qs::set_error(QS_E_HANDLE, "invalid batch handle");
    if (n_regs) *n_regs = b->count;
    if (tile_qubits) *tile_qubits = b->TB + b->RB;
    if (n_passes) *n_passes = b->passes_total;
    return QS_OK;
}


// ---- k-qubit gates and Kraus maps -------------------------------------------
// Sec. II.B.1: the pair update of Eq. 1 generalises to a group of 2^k
// amplitudes for a gate on k qubits, and the Eq. 2 identity holds for
// multi-qubit gates (G on the row qubits, conj(G) on the column qubits); a
// Kraus map is applied through the same identity as its superoperator
// sum_m conj(K_m) (x) K_m on the row and column qubits of its targets.

namespace {

// max |(A A^dagger - I)[r][c]| (d x d, row-major) or, with `kraus`,
// max |(sum_m K_m^dagger K_m - I)[r][c]| over `count` matrices.
double identity_error(const qs_cplx* a, int d, int count, bool kraus)
{
    double worst = 0.0;
    for (int r = 0; r < d; ++r)
        for (int c = 0; c < d; ++c) {
            double re = 0.0, im = 0.0;
            for (int m = 0; m < count; ++m) {
                const qs_cplx* A = a + (size_t)m * d * d;
                for (int s = 0; s < d; ++s) {
                    // unitary: A[r][s] conj(A[c][s]); Kraus: conj(A[s][r]) A[s][c]
                    const qs_cplx x = kraus ? A[s * d + r] : A[r * d + s];
                    const qs_cplx y = kraus ? A[s * d + c] : A[c * d + s];
                    if (kraus) {
                        re += x.re * y.re + x.im * y.im;
                        im += x.re * y.im - x.im * y.re;
                    } else {
                        re += x.re * y.re + x.im * y.im;
                        im += x.im * y.re - x.re * y.im;
                    }
                }
            }
            if (r == c) re -= 1.0;
            worst = std::max(worst, std::max(fabs(re), fabs(im)));
        }
    return worst;
}

qs_status check_finite(const qs_cplx* a, size_t count)
{
    for (size_t k = 0; k < count; ++k)
        if (!isfinite(a[k].re) || !isfinite(a[k].im)) return qs::set_error(QS_E_ARG, "non-finite matrix entry");
    return QS_OK;
}

// Copy a d x d complex matrix (interleaved doubles) into matrix slot `slot`
// (0 or 1) of the register's scratch, in the register's precision, ordered
// on its stream after earlier work; returns the device address.
qs_status upload_matrix(qs_reg r, int slot, const std::vector<double>& m, const void** dev)
{
    char* dst = (char*)(r->scratch + qs::kScratchMatOff) + (size_t)slot * (32 * 32 * 2 * sizeof(double));
    if (r->prec == QS_C128) {
        QS_HIP(hipMemcpyAsync(dst, m.data(), m.size() * sizeof(double), hipMemcpyHostToDevice, r->stream));
    } else {
        std::vector<float> f(m.begin(), m.end());
        QS_HIP(hipMemcpyAsync(dst, f.data(), f.size() * sizeof(float), hipMemcpyHostToDevice, r->stream));
    }
    *dev = dst;
    return QS_OK;
}

qs_status group_launch(qs_reg r, const int* targets, int k, const int* ctrls, int nc, const void* dev_m, int klass)
{
    const qs::Launch L = launch_of(r);
    return qs::profiled(r, klass, [&](int*) {
        return r->prec == QS_C128
                   ? qs::launch_group_gate<double>(L, r->amp, r->nbits, targets, k, ctrls, nc, (const double*)dev_m)
                   : qs::launch_group_gate<float>(L, r->amp, r->nbits, targets, k, ctrls, nc, (const float*)dev_m);
    });
}

}  // namespace

qs_status qs_multi_qubit_unitary(qs_reg r, const int* controls, int n_controls, const int* targets,
                                 int n_targets, const qs_cplx* u)
{
    QS_CHECK_REG(r);
    if (n_targets < 1 || n_targets > 5) return qs::set_error(QS_E_ARG, "1 to 5 target qubits");
    qs_status s = check_qubits(targets, n_targets, r->n, -1, "targets");
    if (s) return s;
    if ((s = check_qubits(controls, n_controls, r->n, -1, "controls"))) return s;
    for (int i = 0; i < n_controls; ++i)
        for (int j = 0; j < n_targets; ++j)
            if (controls[i] == targets[j]) return qs::set_error(QS_E_ARG, "controls: control equals a target");
    if (!u) return qs::set_error(QS_E_ARG, "NULL matrix");
    const int d = 1 << n_targets;
    if ((s = check_finite(u, (size_t)d * d))) return s;
    if (identity_error(u, d, 1, false) > 1e-10) return qs::set_error(QS_E_NOT_UNITARY, "matrix is not unitary");
    std::vector<double> m(2 * d * d);
    for (int i = 0; i < d * d; ++i) {
        m[2 * i] = u[i].re;
        m[2 * i + 1] = u[i].im;
    }
    const void* dm = nullptr;
    if ((s = upload_matrix(r, 0, m, &dm))) return s;
    if ((s = group_launch(r, targets, n_targets, controls, n_controls, dm, QS_K_GATE))) return s;
    if (r->kind != QS_DENSITY) return QS_OK;
    // Eq. 2: conj(U) on the column qubits, controls shifted likewise
    for (int i = 0; i < d * d; ++i) m[2 * i + 1] = -m[2 * i + 1];
    int ct[5], cc[64];
    for (int j = 0; j < n_targets; ++j) ct[j] = targets[j] + r->n;
    for (int j = 0; j < n_controls; ++j) cc[j] = controls[j] + r->n;
    if ((s = upload_matrix(r, 1, m, &dm))) return s;
    return group_launch(r, ct, n_targets, cc, n_controls, dm, QS_K_GATE);
}

qs_status qs_two_qubit_unitary(qs_reg r, int target1, int target2, const qs_cplx u[16])
{
    const int t[2] = {target1, target2};
    return qs_multi_qubit_unitary(r, nullptr, 0, t, 2, u);
}

qs_status qs_circuit_add_two_qubit_unitary(qs_circuit c, int target1, int target2, const qs_cplx u[16])
{
    if (!valid_circ(c)) return qs::set_error(QS_E_HANDLE, "invalid circuit handle");
    const int t[2] = {target1, target2};
    qs_status s = check_qubits(t, 2, 64, -1, "targets");
    if (s) return s;
    if (!u) return qs::set_error(QS_E_ARG, "NULL matrix");
    if ((s = check_finite(u, 16))) return s;
    if (identity_error(u, 4, 1, false) > 1e-10) return qs::set_error(QS_E_NOT_UNITARY, "matrix is not unitary");
    OpRec op{};
    op.kind = 4;
    op.target = target1;
    op.target2 = target2;
    op.m4.resize(32);
    for (int k = 0; k < 16; ++k) {
        op.m4[2 * k] = u[k].re;
        op.m4[2 * k + 1] = u[k].im;
    }
    c->ops.push_back(op);
    return QS_OK;
}

qs_status qs_mix_multi_kraus(qs_reg r, const int* targets, int n_targets, const qs_cplx* ops, int n_ops)
{
    QS_CHECK_REG(r);
    if (r->kind != QS_DENSITY) return qs::set_error(QS_E_KIND, "Kraus maps need a density matrix");
    if (n_targets < 1 || n_targets > 2) return qs::set_error(QS_E_ARG, "1 or 2 target qubits");
    qs_status s = check_qubits(targets, n_targets, r->n, -1, "targets");
    if (s) return s;
    const int d = 1 << n_targets;
    if (n_ops < 1 || n_ops > d * d) return qs::set_error(QS_E_ARG, "1 to 4^k Kraus operators");
    if (!ops) return qs::set_error(QS_E_ARG, "NULL Kraus operators");
    if ((s = check_finite(ops, (size_t)n_ops * d * d))) return s;
    if (identity_error(ops, d, n_ops, true) > 1e-10)
        return qs::set_error(QS_E_NOT_CPTP, "Kraus operators are not trace preserving");
    // S[(a + d b)][(a' + d b')] = sum_m K_m[a][a'] conj(K_m[b][b']): row
    // index a on the targets, column index b on the targets + N
    const int D = d * d;
    std::vector<double> S(2 * D * D, 0.0);
    for (int m = 0; m < n_ops; ++m) {
        const qs_cplx* K = ops + (size_t)m * d * d;
        for (int a = 0; a < d; ++a)
            for (int b = 0; b < d; ++b)
                for (int a2 = 0; a2 < d; ++a2)
                    for (int b2 = 0; b2 < d; ++b2) {
                        const qs_cplx x = K[a * d + a2], y = K[b * d + b2];
                        const size_t e = (size_t)(a + d * b) * D + (a2 + d * b2);
                        S[2 * e] += x.re * y.re + x.im * y.im;
                        S[2 * e + 1] += x.im * y.re - x.re * y.im;
                    }
    }
    int vt[4];
    for (int j = 0; j < n_targets; ++j) {
        vt[j] = targets[j];
        vt[n_targets + j] = targets[j] + r->n;
    }
    const void* dm = nullptr;
    if ((s = upload_matrix(r, 0, S, &dm))) return s;
    return group_launch(r, vt, 2 * n_targets, nullptr, 0, dm, QS_K_DM_CHANNEL);
}

qs_status qs_mix_kraus(qs_reg r, int target, const qs_cplx* ops, int n_ops)
{
    return qs_mix_multi_kraus(r, &target, 1, ops, n_ops);
}

qs_status qs_mix_two_qubit_kraus(qs_reg r, int target1, int target2, const qs_cplx* ops, int n_ops)
{
    const int t[2] = {target1, target2};
    return qs_mix_multi_kraus(r, t, 2, ops, n_ops);
}

// ---- initialisation variants, copies, overlaps, checkpoints -----------------
// Sec. II.B.1: the state is directly readable and writable; these calls
// build common states and read overlaps without copying the state out.

namespace {

// Order `waiter`'s later work after everything already queued on `producer`.
qs_status order_after(hipStream_t waiter, hipStream_t producer)
{
    if (waiter == producer) return QS_OK;
    hipEvent_t ev;
    QS_HIP(hipEventCreateWithFlags(&ev, hipEventDisableTiming));
    hipError_t e = hipEventRecord(ev, producer);
    if (e == hipSuccess) e = hipStreamWaitEvent(waiter, ev, 0);
    (void)hipEventDestroy(ev);
    if (e != hipSuccess) return qs::hip_error(e, "stream ordering");
    return QS_OK;
}

qs_status read_pair(qs_reg r, double out[2])
{
    const double* dev_out = r->scratch + 4 * qs::kReduceBlocks;
    QS_HIP(hipMemcpyAsync(r->host_res, dev_out, 2 * sizeof(double), hipMemcpyDeviceToHost, r->stream));
    qs_status s = sync_stream(r);
    if (s) return s;
    out[0] = r->host_res[0];
    out[1] = r->host_res[1];
    return QS_OK;
}

}  // namespace

qs_status qs_init_plus(qs_reg r)
{
    QS_CHECK_REG(r);
    // state vector: every amplitude 2^(-n/2); density matrix |+><+|: every entry 2^-N
    const double v = r->kind == QS_DENSITY ? ldexp(1.0, -r->n) : 1.0 / sqrt(ldexp(1.0, r->n));
    const qs::Launch L = launch_of(r);
    const uint64_t len = 1ull << r->nbits;
    return qs::profiled(r, QS_K_INIT, [&](int*) {
        return r->prec == QS_C128 ? qs::launch_init_fill<double>(L, r->amp, len, v, 0.0)
                                  : qs::launch_init_fill<float>(L, r->amp, len, v, 0.0);
    });
}

qs_status qs_init_pure_state(qs_reg r, qs_reg pure)
{
    QS_CHECK_REG(r);
    if (!valid_reg(pure)) return qs::set_error(QS_E_HANDLE, "invalid register handle (pure state)");
    if (pure->kind != QS_STATEVEC) return qs::set_error(QS_E_KIND, "the pure state must be a state vector");
    if (pure->n != r->n || pure->prec != r->prec || pure->env->device != r->env->device)
        return qs::set_error(QS_E_ARG, "registers differ in qubits, precision or device");
    if (pure == r) return QS_OK;
    QS_HIP(hipSetDevice(r->env->device));
    qs_status s = order_after(r->stream, pure->stream);
    if (s) return s;
    const qs::Launch L = launch_of(r);
    if (r->kind == QS_STATEVEC) {
        s = qs::profiled(r, QS_K_INIT, [&](int*) {
            return hipMemcpyAsync(r->amp, pure->amp, r->bytes, hipMemcpyDeviceToDevice, r->stream);
        });
    } else {
        s = qs::profiled(r, QS_K_INIT, [&](int*) {
            return r->prec == QS_C128 ? qs::launch_dm_from_pure<double>(L, r->amp, r->n, pure->amp)
                                      : qs::launch_dm_from_pure<float>(L, r->amp, r->n, pure->amp);
        });
    }
    if (s) return s;
    // later work on `pure` waits for this read
    return order_after(pure->stream, r->stream);
}

qs_status qs_clone(qs_reg dst, qs_reg src)
{
    QS_CHECK_REG(dst);
    if (!valid_reg(src)) return qs::set_error(QS_E_HANDLE, "invalid register handle (source)");
    if (src->n != dst->n || src->kind != dst->kind || src->prec != dst->prec ||
        src->env->device != dst->env->device)
        return qs::set_error(QS_E_ARG, "registers differ in shape, precision or device");
    if (src == dst) return QS_OK;
    QS_HIP(hipSetDevice(dst->env->device));
    qs_status s = order_after(dst->stream, src->stream);
    if (s) return s;
    s = qs::profiled(dst, QS_K_INIT, [&](int*) {
        return hipMemcpyAsync(dst->amp, src->amp, dst->bytes, hipMemcpyDeviceToDevice, dst->stream);
    });
    if (s) return s;
    return order_after(src->stream, dst->stream);
}

qs_status qs_calc_inner_product(qs_reg bra, qs_reg ket, qs_cplx* out)
{
    QS_CHECK_REG(bra);
    if (!valid_reg(ket)) return qs::set_error(QS_E_HANDLE, "invalid register handle (ket)");
    if (!out) return qs::set_error(QS_E_ARG, "NULL output");
    if (bra->kind != QS_STATEVEC || ket->kind != QS_STATEVEC)
        return qs::set_error(QS_E_KIND, "inner products need state vectors");
    if (bra->n != ket->n || bra->prec != ket->prec || bra->env->device != ket->env->device)
        return qs::set_error(QS_E_ARG, "registers differ in qubits, precision or device");
    QS_HIP(hipSetDevice(bra->env->device));
    qs_status s = order_after(bra->stream, ket->stream);
    if (s) return s;
    const qs::Launch L = launch_of(bra);
    double* partials = bra->scratch;
    double* dev_out = bra->scratch + 4 * qs::kReduceBlocks;
    s = qs::profiled(bra, QS_K_REDUCE, [&](int*) {
        return bra->prec == QS_C128
                   ? qs::launch_inner_sv<double>(L, bra->amp, ket->amp, bra->nbits, partials, dev_out)
                   : qs::launch_inner_sv<float>(L, bra->amp, ket->amp, bra->nbits, partials, dev_out);
    });
    if (s) return s;
    double v[2];
    if ((s = read_pair(bra, v))) return s;
    out->re = v[0];
    out->im = v[1];
    return QS_OK;
}

qs_status qs_calc_purity(qs_reg r, double* out)
{
    QS_CHECK_REG(r);
    if (!out) return qs::set_error(QS_E_ARG, "NULL output");
    if (r->kind != QS_DENSITY) return qs::set_error(QS_E_KIND, "purity needs a density matrix");
    // Tr(rho^2) = sum_{jk} rho_jk rho_kj = sum_{jk} |rho_jk|^2 for Hermitian
    // rho: the squared norm of the Eq. 2 vector
    const qs::Launch L = launch_of(r);
    double* partials = r->scratch;
    double* dev_out = r->scratch + 4 * qs::kReduceBlocks;
    qs_status s = qs::profiled(r, QS_K_REDUCE, [&](int*) {
        return r->prec == QS_C128 ? qs::launch_prob_sv<double>(L, r->amp, r->nbits, -1, partials, dev_out)
                                  : qs::launch_prob_sv<float>(L, r->amp, r->nbits, -1, partials, dev_out);
    });
    if (s) return s;
    double v[2];
    if ((s = read_pair(r, v))) return s;
    *out = v[0] + v[1];
    return QS_OK;
}

qs_status qs_calc_fidelity(qs_reg r, qs_reg pure, double* out)
{
    QS_CHECK_REG(r);
    if (!valid_reg(pure)) return qs::set_error(QS_E_HANDLE, "invalid register handle (pure state)");
    if (!out) return qs::set_error(QS_E_ARG, "NULL output");
    if (pure->kind != QS_STATEVEC) return qs::set_error(QS_E_KIND, "the pure state must be a state vector");
    if (pure->n != r->n || pure->prec != r->prec || pure->env->device != r->env->device)
        return qs::set_error(QS_E_ARG, "registers differ in qubits, precision or device");
    if (r->kind == QS_STATEVEC) {
        // |<pure|r>|^2
        qs_cplx ip;
        qs_status s = qs_calc_inner_product(pure, r, &ip);
        if (s) return s;
        *out = ip.re * ip.re + ip.im * ip.im;
        return QS_OK;
    }
    QS_HIP(hipSetDevice(r->env->device));
    qs_status s = order_after(r->stream, pure->stream);
    if (s) return s;
    const qs::Launch L = launch_of(r);
    double* partials = r->scratch;
    double* dev_out = r->scratch + 4 * qs::kReduceBlocks;
    s = qs::profiled(r, QS_K_REDUCE, [&](int*) {
        return r->prec == QS_C128 ? qs::launch_fid_dm<double>(L, r->amp, r->n, pure->amp, partials, dev_out)
                                  : qs::launch_fid_dm<float>(L, r->amp, r->n, pure->amp, partials, dev_out);
    });
    if (s) return s;
    double v[2];
    if ((s = read_pair(r, v))) return s;
    *out = v[0];
    return QS_OK;
}

// Checkpoint file: a 64-byte header (magic "QSTATE01", then int32 n, kind,
// prec, 0, uint64 amplitude count, 32 zero bytes) followed by the raw
// amplitudes in the register's precision, little endian.
namespace {

constexpr char kCkptMagic[8] = {'Q', 'S', 'T', 'A', 'T', 'E', '0', '1'};
constexpr size_t kCkptChunk = 64ull << 20;

struct CkptHeader {
    char magic[8];
    int32_t n, kind, prec, zero;
    uint64_t count;
    uint8_t pad[32];
};
static_assert(sizeof(CkptHeader) == 64, "checkpoint header is 64 bytes");

// Two pinned staging buffers: the copy of one chunk overlaps the file
// transfer of the other.
struct Staging {
    void* buf[2] = {nullptr, nullptr};
    hipEvent_t ev[2] = {nullptr, nullptr};
    ~Staging()
    {
        for (int k = 0; k < 2; ++k) {
            if (ev[k]) (void)hipEventDestroy(ev[k]);
            if (buf[k]) (void)hipHostFree(buf[k]);
        }
    }
    qs_status init(size_t bytes)
    {
        for (int k = 0; k < 2; ++k) {
            if (hipHostMalloc(&buf[k], bytes, hipHostMallocDefault) != hipSuccess) {
                (void)hipGetLastError();
                buf[k] = nullptr;
                return qs::set_error(QS_E_OOM, "cannot allocate pinned staging");
            }
            QS_HIP(hipEventCreateWithFlags(&ev[k], hipEventDisableTiming));
        }
        return QS_OK;
    }
};

}  // namespace

qs_status qs_save_state(qs_reg r, const char* path)
{
    QS_CHECK_REG(r);
    if (!path) return qs::set_error(QS_E_ARG, "NULL path");
    QS_HIP(hipSetDevice(r->env->device));
    FILE* f = fopen(path, "wb");
    if (!f) return qs::set_error(QS_E_ARG, std::string("cannot open ") + path + " for writing");
    CkptHeader h;
    memset(&h, 0, sizeof h);
    memcpy(h.magic, kCkptMagic, 8);
    h.n = r->n;
    h.kind = r->kind;
    h.prec = r->prec;
    h.count = 1ull << r->nbits;
    bool ok = fwrite(&h, sizeof h, 1, f) == 1;
    Staging st;
    const size_t chunk = std::min(kCkptChunk, r->bytes);
    qs_status s = ok ? st.init(chunk) : qs::set_error(QS_E_ARG, "checkpoint write failed");
    size_t pending = 0, pend_bytes = 0;
    int k = 0;
    for (size_t off = 0; !s && off < r->bytes; off += chunk, k ^= 1) {
        const size_t nb = std::min(chunk, r->bytes - off);
        hipError_t e = hipMemcpyAsync(st.buf[k], (const char*)r->amp + off, nb, hipMemcpyDeviceToHost, r->stream);
        if (e == hipSuccess) e = hipEventRecord(st.ev[k], r->stream);
        if (e != hipSuccess) {
            s = qs::hip_error(e, "checkpoint copy");
            break;
        }
        if (off > 0) {  // write the previous chunk while this one is copied
            const int j = k ^ 1;
            e = hipEventSynchronize(st.ev[j]);
            if (e != hipSuccess) s = qs::hip_error(e, "checkpoint copy");
            else if (fwrite(st.buf[j], 1, pend_bytes, f) != pend_bytes) s = qs::set_error(QS_E_ARG, "checkpoint write failed");
        }
        pending = 1;
        pend_bytes = nb;
    }
    if (!s && pending) {
        const int j = k ^ 1;
        hipError_t e = hipEventSynchronize(st.ev[j]);
        if (e != hipSuccess) s = qs::hip_error(e, "checkpoint copy");
        else if (fwrite(st.buf[j], 1, pend_bytes, f) != pend_bytes) s = qs::set_error(QS_E_ARG, "checkpoint write failed");
    }
    if (fclose(f) != 0 && !s) s = qs::set_error(QS_E_ARG, "checkpoint close failed");
    return s;
}

qs_status qs_load_state(qs_reg r, const char* path)
{
    QS_CHECK_REG(r);
    if (!path) return qs::set_error(QS_E_ARG, "NULL path");
    FILE* f = fopen(path, "rb");
    if (!f) return qs::set_error(QS_E_ARG, std::string("cannot open ") + path);
    CkptHeader h;
    if (fread(&h, sizeof h, 1, f) != 1 || memcmp(h.magic, kCkptMagic, 8) != 0) {
        fclose(f);
        return qs::set_error(QS_E_ARG, "not a qstate checkpoint");
    }
    if (h.n != r->n || h.kind != r->kind || h.prec != r->prec || h.count != (1ull << r->nbits)) {
        fclose(f);
        return qs::set_error(QS_E_ARG, "checkpoint shape differs from the register");
    }
    fseek(f, 0, SEEK_END);
    const long size = ftell(f);
    if (size < 0 || (uint64_t)size != sizeof h + r->bytes) {
        fclose(f);
        return qs::set_error(QS_E_ARG, "checkpoint is truncated");
    }
    fseek(f, (long)sizeof h, SEEK_SET);
    QS_HIP(hipSetDevice(r->env->device));
    Staging st;
    const size_t chunk = std::min(kCkptChunk, r->bytes);
    qs_status s = st.init(chunk);
    int k = 0;
    bool used[2] = {false, false};
    for (size_t off = 0; !s && off < r->bytes; off += chunk, k ^= 1) {
        const size_t nb = std::min(chunk, r->bytes - off);
        if (used[k]) {  // the copy out of this buffer must have finished
            const hipError_t e = hipEventSynchronize(st.ev[k]);
            if (e != hipSuccess) {
                s = qs::hip_error(e, "checkpoint copy");
                break;
            }
        }
        if (fread(st.buf[k], 1, nb, f) != nb) {
            s = qs::set_error(QS_E_ARG, "checkpoint read failed");
            break;
        }
        hipError_t e = hipMemcpyAsync((char*)r->amp + off, st.buf[k], nb, hipMemcpyHostToDevice, r->stream);
        if (e == hipSuccess) e = hipEventRecord(st.ev[k], r->stream);
        if (e != hipSuccess) s = qs::hip_error(e, "checkpoint copy");
        used[k] = true;
    }
    fclose(f);
    // the staging buffers are freed on return: wait for the copies
    const qs_status s2 = sync_stream(r);
    return s ? s : s2;
}

}  // extern "C"
