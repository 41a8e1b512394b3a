// tmqcd_dslash_noalloc: the operators of tmqcd_dslash with their temporaries
// in a file-scope device array instead of a caller workspace, for callers that
// cannot allocate device memory.  The kernels are those of tmqcd_dslash; only
// the origin of the scratch memory differs.
//
// In host code `scratch` names a host-side stand-in, not device memory: its
// device address is obtained once per device with hipGetSymbolAddress (with
// that device current) and only that address is ever passed to kernels.
#include <hip/hip_runtime.h>

#include <cmath>
#include <cstdint>
#include <mutex>

#include "device.h"
#include "internal.h"
#include "ops.h"
#include "tmqcd.h"

using namespace tmqcd;

namespace {

constexpr int64_t kScratchBytes = TMQCD_NOALLOC_SCRATCH_BYTES;
constexpr int kMaxDevices = 64;

}  // namespace

// Each GPU the library runs on holds its own copy until the process ends.
static __device__ __align__(256) unsigned char scratch[kScratchBytes];

namespace {

std::mutex g_scratch_mutex;
void* g_scratch_ptr[kMaxDevices];   // device address of `scratch` per device, nullptr until resolved

// The device address of this device's scratch array (resolved on the first call
// for the device, with that device current).  hipSuccess or the failing call's error.
hipError_t scratch_for(int dev, void** out) {
    if (dev < 0 || dev >= kMaxDevices) return hipErrorInvalidDevice;
    std::lock_guard<std::mutex> lock(g_scratch_mutex);
    if (g_scratch_ptr[dev] == nullptr) {
        int cur = 0;
        hipError_t e = hipGetDevice(&cur);
        if (e != hipSuccess) return e;
        if (cur != dev && (e = hipSetDevice(dev)) != hipSuccess) return e;
        void* p = nullptr;
        e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
        if (cur != dev) {
            const hipError_t e2 = hipSetDevice(cur);
            if (e == hipSuccess) e = e2;
        }
        if (e != hipSuccess) return e;
        if (p == nullptr) return hipErrorInvalidSymbol;
        g_scratch_ptr[dev] = p;
    }
    *out = g_scratch_ptr[dev];
    return hipSuccess;
}

bool aligned(const void* p, uintptr_t a) { return (reinterpret_cast<uintptr_t>(p) % a) == 0; }
bool overlap(const void* a, int64_t na, const void* b, int64_t nb) {
    const uintptr_t x = reinterpret_cast<uintptr_t>(a), y = reinterpret_cast<uintptr_t>(b);
    return x < y + (uintptr_t)nb && y < x + (uintptr_t)na;
}
int in_sub(int op) {
    if (op == TMQCD_DSLASH_EO) return TMQCD_ODD;
    if (op == TMQCD_M || op == TMQCD_MDAG || op == TMQCD_MDAGM) return TMQCD_FULL;
    return TMQCD_EVEN;
}
int out_sub(int op) {
    if (op == TMQCD_DSLASH_OE) return TMQCD_ODD;
    if (op == TMQCD_M || op == TMQCD_MDAG || op == TMQCD_MDAGM) return TMQCD_FULL;
    return TMQCD_EVEN;
}
bool valid_problem(const tmqcd_problem* p) {
    if (!p) return false;
    int64_t v = 1;
    for (int i = 0; i < 4; ++i) {
        const int d = p->dims[i];
        if (d < 2 || (d & 1)) return false;
        v *= d;
        if (v > (int64_t)1 << 32) return false;
    }
    return std::isfinite(p->kappa) && std::isfinite(p->mu);
}

}  // namespace

extern "C" {

size_t tmqcd_noalloc_scratch_bytes(void) { return (size_t)kScratchBytes; }

int tmqcd_dslash_noalloc(const tmqcd_problem* prob, const void* U_packed, const void* in, void* out, int op, int prec,
                         int recon, int nrhs, void* stream) {
    if (!valid_problem(prob) || op < TMQCD_DSLASH_EO || op > TMQCD_MHATDAGMHAT || prec < TMQCD_F64 ||
        prec > TMQCD_F16 || recon < TMQCD_RECON18 || recon > TMQCD_RECON8 || nrhs < 1 || nrhs > kMaxRhs ||
        !U_packed || !in || !out)
        return TMQCD_EINVAL;
    for (int i = 0; i < 4; ++i)
        if (!std::isfinite(prob->bc[i][0]) || !std::isfinite(prob->bc[i][1])) return TMQCD_EINVAL;
    if (!aligned(U_packed, kAlignBytes) || !aligned(in, kAlignBytes) || !aligned(out, kAlignBytes))
        return TMQCD_EALIGN;
    const Geom g = make_geom(*prob);
    const int64_t fin = field_bytes(g, prec, in_sub(op)), fout = field_bytes(g, prec, out_sub(op));
    if (overlap(in, nrhs * fin, out, nrhs * fout)) return TMQCD_EALIAS;
    const int64_t need = nrhs * dslash_tmp_bytes(g, op, prec);
    if (need > kScratchBytes) return TMQCD_ESCRATCH;   // rejected before any device call
    hipStream_t s = static_cast<hipStream_t>(stream);
    int dev = 0;
    hipError_t e = s ? hipStreamGetDevice(s, &dev) : hipGetDevice(&dev);
    void* ws = nullptr;
    if (e == hipSuccess && need > 0) e = scratch_for(dev, &ws);
    if (e == hipSuccess) {
        const OpCtx c = make_ctx(*prob, prec, recon, U_packed, s);
        e = apply_operator(c, op, in, out, static_cast<char*>(ws), nrhs);
    }
    if (e != hipSuccess) {
        g_last_hip_error = (int)e;
        return TMQCD_EHIP;
    }
    return TMQCD_OK;
}

}  // extern "C"
