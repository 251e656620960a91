// noalloc.hip -- the fluid moments without any allocation, for callers that
// cannot allocate device memory (code under HIP graph capture, serving loops,
// harnesses that forbid it).
//
// pic_moments accumulates the eleven moment channels into a temporary device
// buffer it allocates per call.  pic_moments_noalloc accumulates them into
// `scratch`, a file-scope device array that each GPU holds for the life of
// the process, and writes the finished moments (divided by the node volumes)
// into the caller's device array, asynchronously on the context's stream.
//
// The array's device address on each GPU comes from hipGetSymbolAddress at
// set-up (pic_init, once per device with that device current); host code
// only ever passes that address to kernels.  Every call on one GPU shares the
// array: each call clears the part it uses first, and calls that overlap on
// one GPU (two contexts' streams running at once) race.
#include <mutex>

#include "fp32.h"
#include "pic_internal.h"

using namespace pic;

namespace {

// 32 MiB: the eleven channels of meshes up to 381300 nodes (256 x 1024 has
// 263425).
constexpr long long kScratchDoubles = 4LL << 20;

static __device__ __align__(256) double scratch[kScratchDoubles];

constexpr int kMaxDevices = 64;
std::mutex g_lock;
double* g_ptr[kMaxDevices] = {};

__global__ void kn_zero(double* p, long long n) {
    for (long long t = (long long)blockIdx.x * blockDim.x + threadIdx.x; t < n; t += (long long)gridDim.x * blockDim.x)
        p[t] = 0.0;
}

__global__ void kn_finish(const double* acc, const double* V, long long N, int channels, double* out) {
    const long long n_all = N * channels;
    for (long long t = (long long)blockIdx.x * blockDim.x + threadIdx.x; t < n_all;
         t += (long long)gridDim.x * blockDim.x)
        out[t] = acc[t] / V[t % N];
}

unsigned int grid_of(long long n) {
    const long long g = (n + 255) / 256;
    return (unsigned int)(g < 1 ? 1 : (g > 4096 ? 4096 : g));
}

}  // namespace

namespace pic {

// The scratch array's address on `device` (the current device), looked up
// once per device.
hipError_t noalloc_setup(int device) {
    if (device < 0 || device >= kMaxDevices) return hipErrorInvalidDevice;
    std::lock_guard<std::mutex> guard(g_lock);
    if (g_ptr[device]) return hipSuccess;
    void* p = nullptr;
    const hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
    if (e != hipSuccess) return e;
    g_ptr[device] = (double*)p;
    return hipSuccess;
}

}  // namespace pic

extern "C" pic_status pic_moments_noalloc(pic_ctx* ctx, int k, double* out) {
    const pic_status st = pic_check_instance(ctx, k);
    if (st != PIC_OK) return st;
    if (!out) return pic_fail(ctx, PIC_EINVAL, "out is NULL");
    const long long N = pic_inst_nodes(ctx, k), need = (long long)kMoments * N;
    if (need > kScratchDoubles)
        return pic_fail(ctx, PIC_EINVAL,
                        "mesh of " + std::to_string(N) + " nodes exceeds the allocation-free moments' scratch (" +
                            std::to_string(kScratchDoubles / kMoments) + " nodes)");
    const int dev = pic_device(ctx);
    double* acc = (dev >= 0 && dev < kMaxDevices) ? g_ptr[dev] : nullptr;
    if (!acc) return pic_fail(ctx, PIC_ESTATE, "scratch of the device not set up");
    hipStream_t s = pic_stream(ctx);
    hipLaunchKernelGGL(kn_zero, dim3(grid_of(need)), dim3(256), 0, s, acc, need);
    hipError_t e = hipGetLastError();
    if (e == hipSuccess) {
        const pic_status m = pic_moments_accumulate(ctx, k, acc);
        if (m != PIC_OK) return m;
        hipLaunchKernelGGL(kn_finish, dim3(grid_of(need)), dim3(256), 0, s, acc, pic_inst_volume(ctx, k), N,
                           kMoments, out);
        e = hipGetLastError();
    }
    if (e != hipSuccess) return pic_fail(ctx, PIC_EDEVICE, std::string("moments: ") + hipGetErrorString(e));
    return PIC_OK;
}
