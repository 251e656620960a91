// stream_probe.hip -- streaming-bandwidth probes of the memory access
// patterns of the particle loop (a measurement tool, not part of the
// method): what HBM rate a kernel that only moves the particle loop's bytes
// reaches on this GPU, for the layout the FP32 form uses and for others.
//
// Patterns over n elements (float unless noted), each timed with HIP events:
//   0 copy      float4 in -> float4 out (n/4 vectors; 8 B per element)
//   1 read6     read 5 floats + 1 u64 per element, one sum per workgroup
//   2 write5    write 5 floats per element
//   3 soa       the particle step's traffic: read r, z, vr, vt, vz + u64
//               key, write r, z, vr, vt, vz in place (48 B per element),
//               grid-stride, 256-thread workgroups
//   4 soa_pers  the same in 1024-thread workgroups, two per CU, each taking
//               one contiguous range of 64-element-aligned passes (the
//               particle kernel's static balance)
//   5 aosoa     the same bytes with the seven words of 64 consecutive
//               elements stored together (1792 B per 64 elements)
//   6 aosoa8    eight words per element (the seven and an unread weight),
//               2048 B per 64 elements
//   7 aosoa8_pers  aosoa8 in the particle kernel's launch shape (as 4)
// sp_run returns the average milliseconds per launch over `reps` launches
// after one warm-up launch, or a negative value on a HIP error.
#include <hip/hip_runtime.h>

namespace {

__global__ void sp_copy(const float4* __restrict__ a, float4* __restrict__ b, long long n4) {
    for (long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x; i < n4; i += (long long)gridDim.x * blockDim.x)
        b[i] = a[i];
}

__global__ void sp_read6(const float* __restrict__ r, const float* __restrict__ z, const float* __restrict__ vr,
                         const float* __restrict__ vt, const float* __restrict__ vz,
                         const unsigned long long* __restrict__ key, long long n, float* out) {
    float acc = 0.0f;
    for (long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (long long)gridDim.x * blockDim.x)
        acc += r[i] + z[i] + vr[i] + vt[i] + vz[i] + (float)(key[i] & 1ull);
    __shared__ float s[256];
    s[threadIdx.x] = acc;
    __syncthreads();
    if (threadIdx.x == 0) {
        float t = 0.0f;
        for (int k = 0; k < (int)blockDim.x; ++k) t += s[k];
        out[blockIdx.x] = t;
    }
}

__global__ void sp_write5(float* r, float* z, float* vr, float* vt, float* vz, long long n) {
    for (long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (long long)gridDim.x * blockDim.x) {
        const float x = (float)i;
        r[i] = x; z[i] = x; vr[i] = x; vt[i] = x; vz[i] = x;
    }
}

__device__ __forceinline__ void touch(float& r, float& z, float& vr, float& vt, float& vz, unsigned long long k) {
    const float d = (float)(k & 1ull) * 1e-30f;
    r += vr * 1e-12f;
    z += vz * 1e-12f;
    vr += d;
    vt -= d;
    vz += d;
}

__global__ void sp_soa(float* r, float* z, float* vr, float* vt, float* vz, const unsigned long long* key, long long n) {
    for (long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (long long)gridDim.x * blockDim.x) {
        float a = r[i], b = z[i], c = vr[i], d = vt[i], e = vz[i];
        touch(a, b, c, d, e, key[i]);
        r[i] = a; z[i] = b; vr[i] = c; vt[i] = d; vz[i] = e;
    }
}

__global__ void __launch_bounds__(1024) sp_soa_pers(float* r, float* z, float* vr, float* vt, float* vz,
                                                    const unsigned long long* key, long long n) {
    const long long G = gridDim.x, w = blockIdx.x;
    const long long blocks = (n + 63) / 64;
    const long long b0 = w * blocks / G, b1 = (w + 1) * blocks / G;
    for (long long base = b0 * 64; base < b1 * 64; base += 1024) {
        const long long i = base + threadIdx.x;
        if (i < b1 * 64 && i < n) {
            float a = r[i], b = z[i], c = vr[i], d = vt[i], e = vz[i];
            touch(a, b, c, d, e, key[i]);
            r[i] = a; z[i] = b; vr[i] = c; vt[i] = d; vz[i] = e;
        }
    }
}

// seven 4-byte words per element (r, z, vr, vt, vz, key low, key high),
// 64 elements per block: word f of element i at (i / 64) * 448 + f * 64 + i % 64
__global__ void sp_aosoa(unsigned int* p, long long n) {
    for (long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (long long)gridDim.x * blockDim.x) {
        unsigned int* q = p + (i >> 6) * 448 + (i & 63);
        float a = __uint_as_float(q[0]), b = __uint_as_float(q[64]), c = __uint_as_float(q[128]);
        float d = __uint_as_float(q[192]), e = __uint_as_float(q[256]);
        const unsigned long long k = ((unsigned long long)q[384] << 32) | q[320];
        touch(a, b, c, d, e, k);
        q[0] = __float_as_uint(a); q[64] = __float_as_uint(b); q[128] = __float_as_uint(c);
        q[192] = __float_as_uint(d); q[256] = __float_as_uint(e);
    }
}

// eight words per element: word f of element i at (i / 64) * 512 + f * 64 + i % 64
__device__ __forceinline__ void aosoa8_one(unsigned int* p, long long i) {
    unsigned int* q = p + (i >> 6) * 512 + (i & 63);
    float a = __uint_as_float(q[0]), b = __uint_as_float(q[64]), c = __uint_as_float(q[128]);
    float d = __uint_as_float(q[192]), e = __uint_as_float(q[256]);
    const unsigned long long k = ((unsigned long long)q[384] << 32) | q[320];
    touch(a, b, c, d, e, k);
    q[0] = __float_as_uint(a); q[64] = __float_as_uint(b); q[128] = __float_as_uint(c);
    q[192] = __float_as_uint(d); q[256] = __float_as_uint(e);
}

__global__ void sp_aosoa8(unsigned int* p, long long n) {
    for (long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (long long)gridDim.x * blockDim.x)
        aosoa8_one(p, i);
}

__global__ void __launch_bounds__(1024) sp_aosoa8_pers(unsigned int* p, long long n) {
    const long long G = gridDim.x, w = blockIdx.x;
    const long long blocks = (n + 63) / 64;
    const long long b0 = w * blocks / G, b1 = (w + 1) * blocks / G;
    for (long long base = b0 * 64; base < b1 * 64; base += 1024) {
        const long long i = base + threadIdx.x;
        if (i < b1 * 64 && i < n) aosoa8_one(p, i);
    }
}

// Seven-word blocks in the particle kernel's two launch shapes: U elements
// per lane and pass, 1024-thread workgroups over statically balanced ranges
// of whole blocks (U = 1: two workgroups per CU; U = 2: one, every element's
// loads issued before any element's stores).
template <int U>
__global__ void __launch_bounds__(1024) sp_aosoa_pers(unsigned int* p, long long n) {
    const long long G = gridDim.x, w = blockIdx.x;
    const long long blocks = (n + 63) / 64;
    const long long b0 = w * blocks / G, b1 = (w + 1) * blocks / G;
    const long long end = min(b1 * 64, n);
    for (long long base = b0 * 64; base < end; base += 1024 * U) {
        float a[U], b[U], c[U], d[U], e[U];
        unsigned long long k[U];
        unsigned int* q[U];
        bool in[U];
#pragma unroll
        for (int u = 0; u < U; ++u) {
            const long long i = base + u * 1024 + threadIdx.x;
            in[u] = i < end;
            q[u] = p + ((in[u] ? i : base) >> 6) * 448 + ((in[u] ? i : base) & 63);
            a[u] = __uint_as_float(q[u][0]); b[u] = __uint_as_float(q[u][64]); c[u] = __uint_as_float(q[u][128]);
            d[u] = __uint_as_float(q[u][192]); e[u] = __uint_as_float(q[u][256]);
            k[u] = ((unsigned long long)q[u][384] << 32) | q[u][320];
        }
#pragma unroll
        for (int u = 0; u < U; ++u) {
            touch(a[u], b[u], c[u], d[u], e[u], k[u]);
            if (in[u]) {
                q[u][0] = __float_as_uint(a[u]); q[u][64] = __float_as_uint(b[u]); q[u][128] = __float_as_uint(c[u]);
                q[u][192] = __float_as_uint(d[u]); q[u][256] = __float_as_uint(e[u]);
            }
        }
    }
}

__global__ void sp_fill(unsigned int* p, long long n, unsigned int v) {
    for (long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (long long)gridDim.x * blockDim.x)
        p[i] = v + (unsigned int)(i & 0xff);
}

}  // namespace

extern "C" double sp_run(int pattern, long long n, int reps, double* gbytes) {
    if (n <= 0 || reps <= 0) return -1.0;
    int dev = 0, cus = 0;
    if (hipGetDevice(&dev) != hipSuccess) return -1.0;
    if (hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess) return -1.0;
    // every pattern's buffers: 8 words per element is the largest
    unsigned int* buf = nullptr;
    const size_t words = (size_t)n * 8 + 64 * 512;
    if (hipMalloc(&buf, words * 4) != hipSuccess) return -2.0;
    float* out = nullptr;
    if (hipMalloc(&out, 65536 * 4) != hipSuccess) {
        (void)hipFree(buf);
        return -2.0;
    }
    hipLaunchKernelGGL(sp_fill, dim3(8192), dim3(256), 0, 0, buf, (long long)words, 0x3f000000u);
    float* f = (float*)buf;
    float *r = f, *z = f + n, *vr = f + 2 * n, *vt = f + 3 * n, *vz = f + 4 * n;
    unsigned long long* key = (unsigned long long*)(f + 5 * n + (n & 1));
    const unsigned int grid = (unsigned int)cus * 32;
    double bytes = 0.0;
    auto launch = [&]() {
        switch (pattern) {
            case 0:
                hipLaunchKernelGGL(sp_copy, dim3(grid), dim3(256), 0, 0, (const float4*)f, (float4*)(f + 4 * (n / 4) + 64),
                                   n / 4);
                bytes = 32.0 * (double)(n / 4);
                break;
            case 1:
                hipLaunchKernelGGL(sp_read6, dim3(grid), dim3(256), 0, 0, r, z, vr, vt, vz, key, n, out);
                bytes = 28.0 * (double)n;
                break;
            case 2:
                hipLaunchKernelGGL(sp_write5, dim3(grid), dim3(256), 0, 0, r, z, vr, vt, vz, n);
                bytes = 20.0 * (double)n;
                break;
            case 3:
                hipLaunchKernelGGL(sp_soa, dim3(grid), dim3(256), 0, 0, r, z, vr, vt, vz, key, n);
                bytes = 48.0 * (double)n;
                break;
            case 4:
                hipLaunchKernelGGL(sp_soa_pers, dim3((unsigned int)cus * 2), dim3(1024), 0, 0, r, z, vr, vt, vz, key, n);
                bytes = 48.0 * (double)n;
                break;
            case 5:
                hipLaunchKernelGGL(sp_aosoa, dim3(grid), dim3(256), 0, 0, buf, n);
                bytes = 48.0 * (double)n;
                break;
            case 6:
                hipLaunchKernelGGL(sp_aosoa8, dim3(grid), dim3(256), 0, 0, buf, n);
                bytes = 48.0 * (double)n;
                break;
            case 7:
                hipLaunchKernelGGL(sp_aosoa8_pers, dim3((unsigned int)cus * 2), dim3(1024), 0, 0, buf, n);
                bytes = 48.0 * (double)n;
                break;
            case 8:
                hipLaunchKernelGGL(sp_aosoa_pers<1>, dim3((unsigned int)cus * 2), dim3(1024), 0, 0, buf, n);
                bytes = 48.0 * (double)n;
                break;
            case 9:
                hipLaunchKernelGGL(sp_aosoa_pers<2>, dim3((unsigned int)cus), dim3(1024), 0, 0, buf, n);
                bytes = 48.0 * (double)n;
                break;
            default:
                bytes = -1.0;
        }
    };
    launch();
    double ms = -1.0;
    hipEvent_t e0, e1;
    if (bytes > 0.0 && hipEventCreate(&e0) == hipSuccess && hipEventCreate(&e1) == hipSuccess) {
        (void)hipEventRecord(e0, 0);
        for (int k = 0; k < reps; ++k) launch();
        (void)hipEventRecord(e1, 0);
        if (hipEventSynchronize(e1) == hipSuccess) {
            float t = 0.0f;
            (void)hipEventElapsedTime(&t, e0, e1);
            ms = (double)t / reps;
        }
        (void)hipEventDestroy(e0);
        (void)hipEventDestroy(e1);
    }
    if (hipDeviceSynchronize() != hipSuccess) ms = -3.0;
    (void)hipFree(buf);
    (void)hipFree(out);
    if (gbytes) *gbytes = bytes * 1e-9;
    return ms;
}
