// Bandwidth probes whose ceilings bench.py reports (measurement only, not part of
// the P_N library): what HBM bandwidth this GPU delivers to a flat stream, a
// flat copy, and to a pure-memory kernel with the access pattern of the
// window sweep (256-thread tiles; per step 8 planes read and 4 written, in
// row pieces of one wave's width; planes one grid apart; no arithmetic).
#include <hip/hip_runtime.h>

#include <cstdint>

namespace {

__global__ void k_read_flat(const float4* __restrict__ a, long long n, float* out) {
    const long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) {
        const float4 v = a[i];
        if (v.x + v.y + v.z + v.w == 1234.5f) out[0] = v.x;  // keeps the load alive
    }
}

__global__ void k_copy_flat(const float4* __restrict__ a, float4* __restrict__ b, long long n) {
    const long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) b[i] = a[i];
}

template <class V, int S, int W>
__global__ void k_pattern(const V* __restrict__ in, V* __restrict__ out, long long plane,
                          int nit, int ntile) {
    const int tile = blockIdx.x % ntile;
    const int part = blockIdx.x / ntile;
    const long long off = (long long)tile * 256 + threadIdx.x;
    V acc = V();
    for (int it = 0; it < nit; ++it) {
        const long long pb = ((long long)part * nit + it) * S;
#pragma unroll
        for (int s = 0; s < S; ++s) acc += in[(pb + s) * plane + off];
        const long long wb = ((long long)part * nit + it) * W;
#pragma unroll
        for (int w = 0; w < W; ++w) out[(wb + w) * plane + off] = acc;
    }
}

double timed(hipEvent_t e0, hipEvent_t e1, hipStream_t st, int reps, double bytes,
             void (*launch)(void*), void* arg) {
    launch(arg);
    (void)hipStreamSynchronize(st);
    (void)hipEventRecord(e0, st);
    for (int r = 0; r < reps; ++r) launch(arg);
    (void)hipEventRecord(e1, st);
    (void)hipEventSynchronize(e1);
    float ms = 0;
    (void)hipEventElapsedTime(&ms, e0, e1);
    return bytes * reps / (ms * 1e-3) / 1e9;
}

struct Args {
    void *a, *b;
    float* out;
    long long n;
    hipStream_t st;
    int esz;  // pattern element size: 8 (double) or 4 (float)
    long long ncell;
    int nplanes;
};

void l_read(void* p) {
    Args* g = (Args*)p;
    const long long n4 = g->n / 16;
    hipLaunchKernelGGL(k_read_flat, dim3((unsigned)((n4 + 255) / 256)), dim3(256), 0, g->st,
                       (const float4*)g->a, n4, g->out);
}
void l_copy(void* p) {
    Args* g = (Args*)p;
    const long long n4 = g->n / 16;
    hipLaunchKernelGGL(k_copy_flat, dim3((unsigned)((n4 + 255) / 256)), dim3(256), 0, g->st,
                       (const float4*)g->a, (float4*)g->b, n4);
}
void l_pattern(void* p) {
    Args* g = (Args*)p;
    const int S = 8, parts = 10;
    const int nit = g->nplanes / (S * parts);
    const int ntile = (int)(g->ncell / 256);
    if (g->esz == 8)
        hipLaunchKernelGGL((k_pattern<double, 8, 4>), dim3(ntile * parts), dim3(256), 0, g->st,
                           (const double*)g->a, (double*)g->b, g->ncell, nit, ntile);
    else
        hipLaunchKernelGGL((k_pattern<float, 8, 4>), dim3(ntile * parts), dim3(256), 0, g->st,
                           (const float*)g->a, (float*)g->b, g->ncell, nit, ntile);
}

}  // namespace

extern "C" {

// GB/s of: [0] flat float4 read, [1] flat copy (read + write bytes),
// [2] sweep-pattern FP64, [3] sweep-pattern FP32, over `bytes` of device
// memory per buffer (two buffers are allocated).  Returns 0 or a negative
// HIP error code.  The pattern runs on a grid of `ncell` cells (a multiple
// of 256) with 1600 planes read and 800 written per launch.
int pmp_ceilings(long long bytes, long long ncell, double* gbs) {
    const int nrd = 1600, nwr = 800;
    const long long need = ncell * 8LL * nrd;
    const long long sz = bytes > need ? bytes : need;
    void *a = nullptr, *b = nullptr;
    float* out = nullptr;
    if (hipMalloc(&a, sz) != hipSuccess) return -2;
    if (hipMalloc(&b, sz) != hipSuccess) { (void)hipFree(a); return -2; }
    if (hipMalloc(&out, 64) != hipSuccess) { (void)hipFree(a); (void)hipFree(b); return -2; }
    hipStream_t st;
    (void)hipStreamCreate(&st);
    (void)hipMemsetAsync(a, 0, sz, st);
    (void)hipMemsetAsync(b, 0, sz, st);
    hipEvent_t e0, e1;
    (void)hipEventCreate(&e0);
    (void)hipEventCreate(&e1);
    Args g{a, b, out, bytes, st, 8, ncell, nrd};
    gbs[0] = timed(e0, e1, st, 5, (double)bytes, l_read, &g);
    gbs[1] = timed(e0, e1, st, 5, 2.0 * bytes, l_copy, &g);
    const double pat = (double)ncell * (nrd + nwr);  // elements moved per launch
    g.esz = 8;
    gbs[2] = timed(e0, e1, st, 3, pat * 8, l_pattern, &g);
    g.esz = 4;
    gbs[3] = timed(e0, e1, st, 3, pat * 4, l_pattern, &g);
    const hipError_t err = hipGetLastError();
    (void)hipEventDestroy(e0);
    (void)hipEventDestroy(e1);
    (void)hipStreamDestroy(st);
    (void)hipFree(a);
    (void)hipFree(b);
    (void)hipFree(out);
    return err == hipSuccess ? 0 : -3;
}

}  // extern "C"
