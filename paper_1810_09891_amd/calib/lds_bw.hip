// LDS throughput of one gfx950 device: conflict-free 16-byte and 8-byte reads and 8-byte
// read-add-write, the access patterns of the interpolation and spreading kernels.  Prints
// TB/s and bytes per clock per compute unit.  Every index stays inside the 64 KB array.
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

__global__ __launch_bounds__(kThreads) void rd128(float *out)
{
    __shared__ float4 lds[4096];  // 64 KB
    for (int i = threadIdx.x; i < 4096; i += kThreads)
        lds[i] = make_float4(i, i + 1, i + 2, i + 3);
    __syncthreads();
    float4 acc = make_float4(0, 0, 0, 0);
    for (int it = 0; it < kIters; ++it) {
        const float4 v = lds[(threadIdx.x + it * kThreads) & 4095];
        acc.x += v.x; acc.y += v.y; acc.z += v.z; acc.w += v.w;
    }
    out[blockIdx.x * kThreads + threadIdx.x] = acc.x + acc.y + acc.z + acc.w;
}

__global__ __launch_bounds__(kThreads) void rd64(float *out)
{
    __shared__ float2 lds[8192];  // 64 KB
    for (int i = threadIdx.x; i < 8192; i += kThreads)
        lds[i] = make_float2(i, i + 1);
    __syncthreads();
    float2 acc = make_float2(0, 0);
    for (int it = 0; it < kIters; ++it) {
        const float2 v = lds[(threadIdx.x + it * kThreads) & 8191];
        acc.x += v.x; acc.y += v.y;
    }
    out[blockIdx.x * kThreads + threadIdx.x] = acc.x + acc.y;
}

// read-add-write of 8-byte cells, each lane its own cell (no two lanes share a cell)
__global__ __launch_bounds__(kThreads) void rmw64(float *out)
{
    __shared__ float2 lds[8192];
    for (int i = threadIdx.x; i < 8192; i += kThreads)
        lds[i] = make_float2(0, 0);
    __syncthreads();
    for (int it = 0; it < kIters; ++it) {
        const int idx = (threadIdx.x + (it & 31) * kThreads) & 8191;
        float2 v = lds[idx];
        v.x += 1.f; v.y += 2.f;
        lds[idx] = v;
    }
    __syncthreads();
    out[blockIdx.x * kThreads + threadIdx.x] = lds[threadIdx.x].x;
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
    K ks[] = {{"ds_read_b128", rd128, 16.0}, {"ds_read_b64", rd64, 8.0}, {"rmw_b64", rmw64, 16.0}};
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
        printf("%-14s %.2f TB/s = %.1f B/clk/CU at %d MHz, %d CUs\n", k.name, tbs,
               tbs * 1e12 / (cus * clk * 1e3), clk / 1000, cus);
    }
    CHECK(hipFree(out));
    return 0;
}
