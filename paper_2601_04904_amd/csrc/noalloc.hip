// Batched diagonal-block inverse that allocates nothing: the same kernels as
// bt_si_sq_diag_inverse, with every piece of scratch (job descriptors, the
// device status word, working copies, panel transforms, pivot arrays) taken
// from one file-scope device array of fixed size.  For callers that cannot
// allocate device memory (code under graph capture, tight serving loops).
//
// In host code the array's name is a host-side stand-in, not a device
// address: its device address is looked up once per device with
// hipGetSymbolAddress (with that device current) and only that address is
// handed to kernels.  Each device holds its own copy of the array until the
// process ends; calls on one device share it, so calls that overlap on one
// device race.
#include "../../include/bt_si_sq.h"
#include "../../include/bt_si_sq_diag.h"
#include "common.h"

#include <mutex>
#include <string>

namespace btsq {
hipError_t launch_inverse_sequence(const InvJob* d_jobs, int njobs, int maxd, DevStatus* status,
                                   hipStream_t s);
void set_global_error(const std::string& msg);
}  // namespace btsq

using namespace btsq;

namespace {

constexpr size_t kScratchBytes = (size_t)64 << 20;   // 64 MiB per device
constexpr int kMaxDevices = 64;

__device__ __align__(256) char scratch[kScratchBytes];

std::mutex g_mu;
char* g_scratch[kMaxDevices] = {};

// Device address of this device's scratch array (looked up at the first call
// on the device).
hipError_t scratch_ptr(char** out) {
    int dev = 0;
    hipError_t e = hipGetDevice(&dev);
    if (e != hipSuccess) return e;
    if (dev < 0 || dev >= kMaxDevices) return hipErrorInvalidDevice;
    std::lock_guard<std::mutex> lk(g_mu);
    if (!g_scratch[dev]) {
        void* p = nullptr;
        e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
        if (e != hipSuccess) return e;
        g_scratch[dev] = static_cast<char*>(p);
    }
    *out = g_scratch[dev];
    return hipSuccess;
}

// Layout inside the scratch array: [status | jobs | per-job W, Mm, perm, used].
__host__ __device__ inline size_t jobs_offset() { return 256; }
__host__ __device__ inline size_t pool_offset(int count) {
    return align256(jobs_offset() + (size_t)count * sizeof(InvJob));
}
size_t scratch_need(int d, int count) { return pool_offset(count) + (size_t)count * inv_scratch_bytes(d); }

// Clears the status word and writes the job descriptors (one thread per job):
// job i inverts src + i d^2 into dst + i d^2 with its scratch from the pool.
__global__ void noalloc_setup(char* base, const double2* src, double2* dst, int d, int count) {
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i == 0) {
        DevStatus* st = reinterpret_cast<DevStatus*>(base);
        st->code = 0;
        st->tag = 0;
    }
    if (i >= count) return;
    InvJob j{};
    j.src = src + (size_t)i * d * d;
    j.dst = dst + (size_t)i * d * d;
    j.d = d;
    j.tag = i;
    inv_bind_scratch(j, base, pool_offset(count) + (size_t)i * inv_scratch_bytes(d), d);
    reinterpret_cast<InvJob*>(base + jobs_offset())[i] = j;
}

}  // namespace

extern "C" size_t bt_si_sq_diag_inverse_noalloc_max_bytes(void) { return kScratchBytes; }

extern "C" bt_status bt_si_sq_diag_inverse_noalloc(const void* src, void* dst, int32_t d, int32_t count,
                                                   int32_t* bad_index, void* hip_stream) {
    if (bad_index) *bad_index = -1;
    if (!src || !dst || d < 1 || d > kInvMaxDim || count < 0) {
        set_global_error("diag_inverse_noalloc: bad arguments (1 <= d <= 1024)");
        return BT_ERR_INVALID;
    }
    if (count == 0) return BT_OK;
    const size_t need = scratch_need(d, count);
    if (need > kScratchBytes) {
        set_global_error("diag_inverse_noalloc: " + std::to_string(count) + " inverses of size " +
                         std::to_string(d) + " need " + std::to_string(need) + " bytes of scratch, above the " +
                         std::to_string(kScratchBytes) + " bytes of the fixed array");
        return BT_ERR_INVALID;
    }
    hipStream_t s = reinterpret_cast<hipStream_t>(hip_stream);
    char* base = nullptr;
    hipError_t e = scratch_ptr(&base);
    if (e != hipSuccess) {
        set_global_error(std::string("diag_inverse_noalloc: hipGetSymbolAddress: ") + hipGetErrorString(e));
        return BT_ERR_HIP;
    }
    DevStatus* status = reinterpret_cast<DevStatus*>(base);
    const InvJob* jobs = reinterpret_cast<const InvJob*>(base + jobs_offset());
    hipLaunchKernelGGL(noalloc_setup, dim3((count + 255) / 256), dim3(256), 0, s, base,
                       reinterpret_cast<const double2*>(src), reinterpret_cast<double2*>(dst), d, count);
    e = hipGetLastError();
    if (e == hipSuccess) e = launch_inverse_sequence(jobs, count, d, status, s);
    hipError_t e2 = hipStreamSynchronize(s);
    DevStatus out{0, 0};
    if (e == hipSuccess && e2 == hipSuccess) e2 = hipMemcpy(&out, status, sizeof out, hipMemcpyDeviceToHost);
    if (e != hipSuccess || e2 != hipSuccess) {
        set_global_error(std::string("diag_inverse_noalloc: ") + hipGetErrorString(e != hipSuccess ? e : e2));
        return BT_ERR_HIP;
    }
    if (out.code != 0) {
        if (bad_index) *bad_index = out.tag;
        set_global_error("diag_inverse_noalloc: singular or non-finite pivot");
        return BT_ERR_SINGULAR;
    }
    return BT_OK;
}
