// An entry point that allocates no device memory: the affine-projection
// adjoint with its staging buffers (the x and y of the KKT solve applied to
// the cotangent) in a fixed file-scope device array instead of buffers the
// handle allocates at its first differentiation call.  For callers that may
// not allocate (code under HIP graph capture, serving loops).
//
// The array is a static __device__ symbol: each device the library runs on
// holds its own copy for the life of the process.  Its device address is
// looked up once per device (hipGetSymbolAddress, with that device current)
// at the entry point's first call there and kept; host code uses that
// address, never the symbol's host-side name.  Calls on one device share the
// array, so calls that overlap on one device race.  Every element the
// kernels read is written earlier in the same call, so nothing needs
// clearing between calls.
#include <map>
#include <mutex>

#include "cdcs_internal.h"

namespace {

constexpr int64_t kScratchX = int64_t(1) << 20;  // solve output x: ldU <= 2^20 entries
constexpr int64_t kScratchY = 8192;              // solve output y: ldM <= 8192 rows
constexpr int64_t kScratchDoubles = kScratchX + kScratchY;  // 8,454,144 bytes

__device__ __align__(256) double scratch[kScratchDoubles];

std::mutex g_scratch_mu;
std::map<int, double *> g_scratch_ptr;  // device -> address of its copy of `scratch`

cdcs_status scratch_on_current_device(double **out) {
    int dev = 0;
    hipError_t e = hipGetDevice(&dev);
    if (e != hipSuccess) return cdcs::set_error(CDCS_E_DEVICE, std::string("hipGetDevice: ") + hipGetErrorString(e));
    std::lock_guard<std::mutex> lock(g_scratch_mu);
    auto it = g_scratch_ptr.find(dev);
    if (it != g_scratch_ptr.end()) {
        *out = it->second;
        return CDCS_OK;
    }
    void *p = nullptr;
    e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
    if (e != hipSuccess || p == nullptr)
        return cdcs::set_error(CDCS_E_DEVICE, std::string("hipGetSymbolAddress(scratch): ") + hipGetErrorString(e));
    g_scratch_ptr[dev] = static_cast<double *>(p);
    *out = static_cast<double *>(p);
    return CDCS_OK;
}

}  // namespace

extern "C" cdcs_status cdcs_affine_project_adjoint_noalloc(cdcs_handle *h, const double *xbar, double *r1bar,
                                                          double *r2bar, hipStream_t stream) {
    if (!h || !xbar || !r1bar || !r2bar) return cdcs::set_error(CDCS_E_ARG, "NULL argument");
    int64_t ldU = 0, ldM = 0;
    cdcs::handle_dims(h, &ldU, &ldM);
    if (ldU > kScratchX || ldM > kScratchY)
        return cdcs::set_error(CDCS_E_ARG, "handle too large for the fixed scratch (entries padded to " +
                                               std::to_string(ldU) + " > " + std::to_string(kScratchX) +
                                               " or constraints padded to " + std::to_string(ldM) + " > " +
                                               std::to_string(kScratchY) + ")");
    double *base = nullptr;
    const cdcs_status st = scratch_on_current_device(&base);
    if (st != CDCS_OK) return st;
    return cdcs::affine_adjoint_into(h, xbar, r1bar, r2bar, base, base + kScratchX, stream);
}
