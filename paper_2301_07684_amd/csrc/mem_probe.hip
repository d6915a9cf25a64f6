// Memory-only reference for the streaming kernel's access pattern (a measurement aid of the
// benchmark, not part of the step's C ABI in include/sfq.h).
//
// Ten FP64 arrays of n elements are read and the last of them written back, as the streaming
// kernel reads p, E, B and the optical depth and writes the depth, with no arithmetic beyond a
// sum that keeps the loads live: 88 bytes per element.  Persistent blocks of 256 threads take
// chunks from a counter; each lane takes `particles_per_lane` adjacent elements per iteration
// with 16-byte non-temporal accesses, all loads of an iteration issued together.  The rate it
// reaches is the practical ceiling of that pattern on the machine, beside the published 8 TB/s.
//
//   int sfq_probe_stream(int blocks_per_cu, int particles_per_lane, uint32_t n, uint32_t chunk,
//                        int repeats, float* median_ms)
//
// blocks_per_cu in [1, 16]; particles_per_lane 2 or 4; chunk a multiple of 256 x
// particles_per_lane; n a positive multiple of chunk; repeats in [3, 1000].  The call allocates
// its arrays (n x 80 bytes) and a 512 MiB pair of buffers whose copy evicts the caches before
// every launch, times `repeats` launches with HIP events on the null stream, frees everything
// and writes the median launch time in ms.  Returns 0, -1 for an argument out of range, or the
// HIP error code of the first call that failed.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cstdint>
#include <vector>

namespace {

typedef double dv2 __attribute__((ext_vector_type(2)));

struct ProbeArrays {
    const double* in[10];
    double* out;
};

template <typename T>
__device__ __forceinline__ T ld_nt(const T* p)
{
    return __builtin_nontemporal_load((const __attribute__((address_space(1))) T*)p);
}
template <typename T>
__device__ __forceinline__ void st_nt(T* p, T v)
{
    __builtin_nontemporal_store(v, (__attribute__((address_space(1))) T*)p);
}

template <int PPL>
__global__ __launch_bounds__(256) void probe_kernel(ProbeArrays A, uint32_t nchunks,
                                                    uint32_t chunk, unsigned* next)
{
    __shared__ unsigned s_c;
    for (;;) {
        if (threadIdx.x == 0) s_c = atomicAdd(next, 1u);
        __syncthreads();
        const unsigned c = s_c;
        __syncthreads();  // every thread has read s_c before thread 0 overwrites it
        if (c >= nchunks) break;
        const size_t start = (size_t)c * chunk;
        for (uint32_t o0 = 0; o0 < chunk; o0 += PPL * 256u) {
            const size_t o = start + o0 + (size_t)PPL * threadIdx.x;
            dv2 v[10][PPL / 2];
#pragma unroll
            for (int k = 0; k < 10; ++k)
#pragma unroll
                for (int h = 0; h < PPL / 2; ++h) v[k][h] = ld_nt((const dv2*)(A.in[k] + o) + h);
#pragma unroll
            for (int h = 0; h < PPL / 2; ++h) {
                dv2 s = v[0][h];
#pragma unroll
                for (int k = 1; k < 10; ++k) s = s * 0.5 + v[k][h];
                st_nt((dv2*)(A.out + o) + h, s);
            }
        }
    }
}

}  // namespace

extern "C" int sfq_probe_stream(int blocks_per_cu, int particles_per_lane, uint32_t n,
                                uint32_t chunk, int repeats, float* median_ms)
{
    if (!median_ms || blocks_per_cu < 1 || blocks_per_cu > 16 || repeats < 3 || repeats > 1000 ||
        (particles_per_lane != 2 && particles_per_lane != 4) || chunk == 0 ||
        chunk % (256u * (uint32_t)particles_per_lane) != 0 || n == 0 || n % chunk != 0)
        return -1;
    int dev = 0, cus = 0;
    hipError_t e = hipGetDevice(&dev);
    if (e == hipSuccess) e = hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev);
    if (e != hipSuccess) return (int)e;
    std::vector<double*> arrays(10, nullptr);
    unsigned* next = nullptr;
    char *flush_a = nullptr, *flush_b = nullptr;
    hipEvent_t e0 = nullptr, e1 = nullptr;
    const size_t bytes = (size_t)n * sizeof(double), flush = (size_t)512 << 20;
    std::vector<float> ms;
    for (int k = 0; k < 10 && e == hipSuccess; ++k) {
        e = hipMalloc(&arrays[k], bytes);
        if (e == hipSuccess) e = hipMemset(arrays[k], 0, bytes);
    }
    if (e == hipSuccess) e = hipMalloc(&next, 64);
    if (e == hipSuccess) e = hipMalloc(&flush_a, flush);
    if (e == hipSuccess) e = hipMalloc(&flush_b, flush);
    if (e == hipSuccess) e = hipEventCreate(&e0);
    if (e == hipSuccess) e = hipEventCreate(&e1);
    if (e == hipSuccess) {
        ProbeArrays A;
        for (int k = 0; k < 10; ++k) A.in[k] = arrays[k];
        A.out = arrays[9];
        const uint32_t nchunks = n / chunk;
        const dim3 grid((unsigned)(cus * blocks_per_cu)), block(256);
        for (int r = 0; r < repeats && e == hipSuccess; ++r) {
            e = hipMemcpy(flush_b, flush_a, flush, hipMemcpyDeviceToDevice);
            if (e == hipSuccess) e = hipMemset(next, 0, 64);
            if (e == hipSuccess) e = hipDeviceSynchronize();
            if (e == hipSuccess) e = hipEventRecord(e0, nullptr);
            if (e != hipSuccess) break;
            if (particles_per_lane == 2)
                hipLaunchKernelGGL(probe_kernel<2>, grid, block, 0, nullptr, A, nchunks, chunk, next);
            else
                hipLaunchKernelGGL(probe_kernel<4>, grid, block, 0, nullptr, A, nchunks, chunk, next);
            e = hipGetLastError();
            if (e == hipSuccess) e = hipEventRecord(e1, nullptr);
            if (e == hipSuccess) e = hipEventSynchronize(e1);
            float t = 0.0f;
            if (e == hipSuccess) e = hipEventElapsedTime(&t, e0, e1);
            if (e == hipSuccess) ms.push_back(t);
        }
    }
    if (e0) (void)hipEventDestroy(e0);
    if (e1) (void)hipEventDestroy(e1);
    if (flush_b) (void)hipFree(flush_b);
    if (flush_a) (void)hipFree(flush_a);
    if (next) (void)hipFree(next);
    for (double* a : arrays)
        if (a) (void)hipFree(a);
    if (e != hipSuccess) return (int)e;
    std::sort(ms.begin(), ms.end());
    *median_ms = ms[ms.size() / 2];
    return 0;
}
