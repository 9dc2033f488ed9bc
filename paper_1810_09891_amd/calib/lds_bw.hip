// LDS throughput of one gfx950 device: conflict-free 16-byte and 8-byte reads and 8-byte
// read-add-write, the access patterns of the interpolation and spreading kernels.  Prints
// TB/s and bytes per clock per compute unit.  Every index stays inside its 32 KB array.
#include <hip/hip_runtime.h>
#include <cstdio>

#define CHECK(x)                                                                                       \
    do {                                                                                               \
        if ((x) != hipSuccess) {                                                                       \
            std::fprintf(stderr, "HIP error at %s:%d\n", __FILE__, __LINE__);                          \
            return 1;                                                                                  \
        }                                                                                              \
    } while (0)
constexpr int kThreads = 256;
constexpr int kIters = 4096;

// Each thread keeps kIndep (kIndep8) independent accesses in flight per iteration (separate
// accumulators), so the figures are LDS throughput rather than the latency of one chain.
constexpr int kIndep = 8;    // 16-byte reads
constexpr int kIndep8 = 16;  // 8-byte reads and read-add-writes

// 8-byte LDS read issued as a relaxed atomic load, the form the window kernels use: it is
// never fused with a neighbour into ds_read2_b64 / ds_read2st64_b64.
__device__ __forceinline__ float2 ld8(float2 *p)
{
    const unsigned long long u = __hip_atomic_load(reinterpret_cast<unsigned long long *>(p), __ATOMIC_RELAXED,
                                                   __HIP_MEMORY_SCOPE_WORKGROUP);
    return __builtin_bit_cast(float2, u);
}

__global__ __launch_bounds__(kThreads) void rd128(float *out)
{
    __shared__ float4 lds[2048];  // 32 KB: five workgroups fit on a compute unit
    for (int i = threadIdx.x; i < 2048; i += kThreads)
        lds[i] = make_float4(i, i + 1, i + 2, i + 3);
    __syncthreads();
    float4 acc[kIndep];
#pragma unroll
    for (int k = 0; k < kIndep; ++k)
        acc[k] = make_float4(0, 0, 0, 0);
    for (int it = 0; it < kIters; it += kIndep) {
#pragma unroll
        for (int k = 0; k < kIndep; ++k) {
            const float4 v = lds[(threadIdx.x + (it + k) * kThreads) & 2047];
            acc[k].x += v.x; acc[k].y += v.y; acc[k].z += v.z; acc[k].w += v.w;
        }
        // every iteration reads the same addresses: a compiler-only memory barrier keeps
        // the loads inside the loop (it emits no instruction)
        asm volatile("" ::: "memory");
    }
    float r = 0;
#pragma unroll
    for (int k = 0; k < kIndep; ++k)
        r += acc[k].x + acc[k].y + acc[k].z + acc[k].w;
    out[blockIdx.x * kThreads + threadIdx.x] = r;
}

__global__ __launch_bounds__(kThreads) void rd64(float *out)
{
    __shared__ float2 lds[4096];  // 32 KB
    for (int i = threadIdx.x; i < 4096; i += kThreads)
        lds[i] = make_float2(i, i + 1);
    __syncthreads();
    float2 acc[kIndep8];
#pragma unroll
    for (int k = 0; k < kIndep8; ++k)
        acc[k] = make_float2(0, 0);
    for (int it = 0; it < kIters; it += kIndep8) {
#pragma unroll
        for (int k = 0; k < kIndep8; ++k) {
            const float2 v = ld8(&lds[(threadIdx.x + (it + k) * kThreads) & 4095]);
            acc[k].x += v.x; acc[k].y += v.y;
        }
    }
    float r = 0;
#pragma unroll
    for (int k = 0; k < kIndep8; ++k)
        r += acc[k].x + acc[k].y;
    out[blockIdx.x * kThreads + threadIdx.x] = r;
}

// read-add-write of 8-byte cells, each lane its own cells (no two lanes share a cell);
// the kIndep8 cells of one iteration are read together, then written
__global__ __launch_bounds__(kThreads) void rmw64(float *out)
{
    __shared__ float2 lds[4096];  // 32 KB
    for (int i = threadIdx.x; i < 4096; i += kThreads)
        lds[i] = make_float2(0, 0);
    __syncthreads();
    for (int it = 0; it < kIters; it += kIndep8) {
        float2 v[kIndep8];
#pragma unroll
        for (int k = 0; k < kIndep8; ++k)
            v[k] = ld8(&lds[(threadIdx.x + ((it + k) & 15) * kThreads) & 4095]);
#pragma unroll
        for (int k = 0; k < kIndep8; ++k) {
            v[k].x += 1.f; v[k].y += 2.f;
            lds[(threadIdx.x + ((it + k) & 15) * kThreads) & 4095] = v[k];
        }
    }
    __syncthreads();
    out[blockIdx.x * kThreads + threadIdx.x] = lds[threadIdx.x].x;
}

// Pairs of adjacent 8-byte reads (a complex64 stencil row read two entries at a time), each
// lane at its own slot: FUSED lets the compiler merge each pair into one ds_read2_b64, else
// the pair is two relaxed-atomic ds_read_b64.  SCATTER places the lanes' slots by a hash
// (stencil rows of unsorted nodes), else lane l reads slot l (conflict-free).
template <bool FUSED, bool SCATTER>
__global__ __launch_bounds__(kThreads) void pair64(float *out)
{
    __shared__ float2 lds[4096];  // 32 KB
    for (int i = threadIdx.x; i < 4096; i += kThreads)
        lds[i] = make_float2(i, i + 1);
    __syncthreads();
    const unsigned lane = threadIdx.x & 63;
    const int s = SCATTER ? (int)(((lane + 1u) * 2654435761u) >> 21) : (int)lane;  // < 2048
    float2 acc[8];
#pragma unroll
    for (int k = 0; k < 8; ++k)
        acc[k] = make_float2(0, 0);
    for (int it = 0; it < kIters; it += 8) {
#pragma unroll
        for (int k = 0; k < 8; ++k) {
            const int a = s + ((it + k) & 15) * 128;  // a + 1 < 2048 + 1921 < 4096
            float2 v, w;
            if (FUSED) {
                v = lds[a];
                w = lds[a + 1];
            } else {
                v = ld8(&lds[a]);
                w = ld8(&lds[a + 1]);
            }
            acc[k].x += v.x * w.x;
            acc[k].y += v.y * w.y;
        }
        asm volatile("" ::: "memory");  // keeps the plain loads inside the loop
    }
    float r = 0;
#pragma unroll
    for (int k = 0; k < 8; ++k)
        r += acc[k].x + acc[k].y;
    out[blockIdx.x * kThreads + threadIdx.x] = r;
}

int main()
{
    int dev = 0, cus = 0, clk = 0;
    CHECK(hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev));
    CHECK(hipDeviceGetAttribute(&clk, hipDeviceAttributeClockRate, dev));  // kHz
    const int blocks = cus * 8;
    float *out;
    CHECK(hipMalloc(&out, sizeof(float) * blocks * kThreads));
    hipEvent_t a, b;
    CHECK(hipEventCreate(&a));
    CHECK(hipEventCreate(&b));
    struct K { const char *name; void (*fn)(float *); double bytes_per_iter; };
    K ks[] = {{"ds_read_b128", rd128, 16.0},
              {"ds_read_b64", rd64, 8.0},
              {"rmw_b64", rmw64, 16.0},
              {"pair read2_b64 seq", pair64<true, false>, 16.0},
              {"pair 2x b64 seq", pair64<false, false>, 16.0},
              {"pair read2_b64 hash", pair64<true, true>, 16.0},
              {"pair 2x b64 hash", pair64<false, true>, 16.0}};
    for (auto &k : ks) {
        hipLaunchKernelGGL(k.fn, dim3(blocks), dim3(kThreads), 0, 0, out);
        CHECK(hipGetLastError());
        CHECK(hipEventRecord(a));
        for (int r = 0; r < 5; ++r)
            hipLaunchKernelGGL(k.fn, dim3(blocks), dim3(kThreads), 0, 0, out);
        CHECK(hipEventRecord(b));
        CHECK(hipEventSynchronize(b));
        float ms = 0;
        CHECK(hipEventElapsedTime(&ms, a, b));
        const double bytes = 5.0 * blocks * kThreads * (double)kIters * k.bytes_per_iter;
        const double tbs = bytes / (ms * 1e-3) / 1e12;
        printf("%-20s %.2f TB/s = %.1f B/clk/CU at %d MHz, %d CUs\n", k.name, tbs,
               tbs * 1e12 / (cus * clk * 1e3), clk / 1000, cus);
    }
    CHECK(hipFree(out));
    return 0;
}
