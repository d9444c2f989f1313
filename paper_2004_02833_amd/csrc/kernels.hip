// HIP kernels of libpm for gfx950 (MI355X).
//
// State layout in HBM: moment-major planes, u[slot][z][y][x] with x fastest;
// slots are grouped by staggered grid (G111, G221, G212, G122 | G211, G121,
// G112, G222) so that each parity is one contiguous range.  One lane owns
// one cell; a wave of 64 lanes covers 64 consecutive cells, so every plane
// access of a wave is a contiguous 256 B (fp32) or 512 B (fp64) segment.
#include <hip/hip_runtime.h>

#include <cmath>
#include <cstdint>

#include "kernels.h"

namespace pm {

// ---------------------------------------------------------------- storage --

struct bf16s {
    uint16_t b;
};

template <class T> struct Acc;
template <> struct Acc<double> { using type = double; };
template <> struct Acc<float> { using type = float; };
template <> struct Acc<bf16s> { using type = float; };

__device__ __forceinline__ double ld(const double* p) { return *p; }
__device__ __forceinline__ float ld(const float* p) { return *p; }
__device__ __forceinline__ float ld(const bf16s* p) {
    return __uint_as_float((uint32_t)p->b << 16);
}

// Round-to-nearest-even conversions from the float64 update.
__device__ __forceinline__ void st(double* p, double v) { *p = v; }
__device__ __forceinline__ void st(float* p, double v) { *p = (float)v; }
__device__ __forceinline__ void st(bf16s* p, double v) {
    float f = (float)v;
    uint32_t x = __float_as_uint(f);
    uint16_t r;
    if ((x & 0x7fffffffu) > 0x7f800000u)
        r = (uint16_t)((x >> 16) | 0x40u);  // quiet NaN
    else
        r = (uint16_t)((x + 0x7fffu + ((x >> 16) & 1u)) >> 16);
    p->b = r;
}

// ---------------------------------------------------------------- indexing --

struct Nbr {
    long long c;
    int off[6];  // +x -x +y -y +z -z, periodic
};

__device__ __forceinline__ Nbr neighbours(long long c, const GridDesc& g) {
    Nbr n;
    n.c = c;
    const long long nxy = (long long)g.nx * g.ny;
    const int z = (int)(c / nxy);
    const long long rem = c - (long long)z * nxy;
    const int y = (int)(rem / g.nx);
    const int x = (int)(rem - (long long)y * g.nx);
    n.off[0] = (x + 1 == g.nx) ? -(g.nx - 1) : 1;
    n.off[1] = (x == 0) ? (g.nx - 1) : -1;
    n.off[2] = (y + 1 == g.ny) ? -(g.ny - 1) * g.nx : g.nx;
    n.off[3] = (y == 0) ? (g.ny - 1) * g.nx : -g.nx;
    n.off[4] = (z + 1 == g.nz) ? (int)(-(long long)(g.nz - 1) * nxy) : (int)nxy;
    n.off[5] = (z == 0) ? (int)((long long)(g.nz - 1) * nxy) : (int)(-nxy);
    return n;
}

__device__ __forceinline__ int pick(const Nbr& n, int code) {
    // Branch-free select of one of six offsets (code is wave-uniform).
    int o = n.off[0];
    o = code == 1 ? n.off[1] : o;
    o = code == 2 ? n.off[2] : o;
    o = code == 3 ? n.off[3] : o;
    o = code == 4 ? n.off[4] : o;
    o = code == 5 ? n.off[5] : o;
    return o;
}

// ------------------------------------------------------------------ tables --
// Per cell: for every grid, the coefficient c on the grid's point (mean of
// sigma_a + sigma_s over the cells sharing it), then alpha = exp(-c tau) and
// beta = tau E(-c tau) = -expm1(-c tau)/c (tau for c = 0), with tau = dt/2
// on odd grids and dt on even grids (eq. (5), (6)).  Moment 0 uses
// c = sigma_a on G111.  Row 18 holds q.

__constant__ int c_grid_bits[8] = {0, 3, 5, 6, 1, 2, 4, 7};

__device__ __forceinline__ void decay(double c, double tau, double& a, double& b) {
    a = exp(-c * tau);
    b = (c == 0.0) ? tau : -expm1(-c * tau) / c;
}

// Cell k + b (b in {0,1}^3, sign +1) or k - b (sign -1), periodic.
__device__ __forceinline__ long long shifted(long long c, int bx, int by, int bz, bool minus,
                                             const GridDesc& g) {
    long long k = c;
    if (bx) k += neighbours(k, g).off[minus ? 1 : 0];
    if (by) k += neighbours(k, g).off[minus ? 3 : 2];
    if (bz) k += neighbours(k, g).off[minus ? 5 : 4];
    return k;
}

// Coefficient of set s (grid order 0..7, or 8 = moment 0) on the point that
// cell c owns: mean of sigma_a (+ sigma_s for s < 8) over the cells sharing it.
__device__ __forceinline__ double cbar_at(const double* __restrict__ sa,
                                          const double* __restrict__ ss, long long c, int s,
                                          const GridDesc& g) {
    if (s == 8) return sa[c];
    const int bits = c_grid_bits[s];
    const int ox = bits & 1, oy = (bits >> 1) & 1, oz = (bits >> 2) & 1;
    double acc = 0.0;
    int cnt = 0;
    for (int bz = 0; bz <= oz; ++bz)
        for (int by = 0; by <= oy; ++by)
            for (int bx = 0; bx <= ox; ++bx) {
                const long long k = shifted(c, bx, by, bz, false, g);
                acc += sa[k] + ss[k];
                ++cnt;
            }
    return acc / cnt;
}

__device__ __forceinline__ double set_tau(int s, double dt) {
    const int bits = s < 8 ? c_grid_bits[s] : 0;
    return (__popc(bits) & 1) ? 0.5 * dt : dt;
}

__global__ void k_tables(const double* __restrict__ sa, const double* __restrict__ ss,
                         const double* __restrict__ q, double* __restrict__ tab, GridDesc g,
                         double dt) {
    const long long c = (long long)blockIdx.x * blockDim.x + threadIdx.x;
    if (c >= g.ncell) return;
    for (int s = 0; s < 9; ++s) {
        double a, b;
        decay(cbar_at(sa, ss, c, s, g), set_tau(s, dt), a, b);
        const int row = s < 8 ? 2 * s : kTabMom0;
        tab[(long long)row * g.ncell + c] = a;
        tab[(long long)(row + 1) * g.ncell + c] = b;
    }
    tab[(long long)kTabQ * g.ncell + c] = q ? q[c] : 0.0;
}

hipError_t launch_tables(const double* sa, const double* ss, const double* q, double* tab,
                         GridDesc g, double dt, hipStream_t st) {
    const int B = 256;
    const long long nb = (g.ncell + B - 1) / B;
    hipLaunchKernelGGL(k_tables, dim3((unsigned)nb), dim3(B), 0, st, sa, ss, q, tab, g, dt);
    return hipGetLastError();
}

// ------------------------------------------------------------ gather sweep --
// Substep S^p_tau of eq. (4)-(5) for every target moment of one parity:
//   r_i = q_i - sum_e K_e (u_src[c + nb_e] - u_src[c]),
//   u_i <- alpha u_i + beta r_i        (float64, rounded to the storage type)
// Sources are the dual parity, which this launch never writes, and every
// target reads only its own old value, so the update is in place.

template <class T>
__global__ void __launch_bounds__(256) k_sweep_gather(T* __restrict__ u,
                                                      const double* __restrict__ tab,
                                                      Schedule s, GridDesc g) {
    using A = typename Acc<T>::type;
    const long long c = (long long)blockIdx.x * blockDim.x + threadIdx.x;
    if (c >= g.ncell) return;
    const Nbr n = neighbours(c, g);
    for (int t = 0; t < s.nrows; ++t) {
        const SweepRow R = s.rows[t];
        A acc = 0;
        for (int e = R.begin; e < R.end; ++e) {
            const SweepEnt E = s.ents[e];
            const T* uj = u + (long long)E.slot * g.pstride;
            const A d = (A)ld(uj + c + pick(n, E.nb)) - (A)ld(uj + c);
            acc += (A)E.K * d;
        }
        const double alpha = tab[(long long)R.tab * g.ncell + c];
        const double beta = tab[(long long)(R.tab + 1) * g.ncell + c];
        const double q = (R.tab == kTabMom0) ? tab[(long long)kTabQ * g.ncell + c] : 0.0;
        T* ut = u + (long long)R.slot * g.pstride + c;
        st(ut, alpha * (double)ld(ut) + beta * (q - (double)acc));
    }
}

hipError_t launch_sweep(int prec, void* u, const double* tab, Schedule s, GridDesc g,
                        hipStream_t st) {
    const int B = 256;
    const unsigned nb = (unsigned)((g.ncell + B - 1) / B);
    switch (prec) {
        case kF64:
            hipLaunchKernelGGL(k_sweep_gather<double>, dim3(nb), dim3(B), 0, st, (double*)u, tab, s, g);
            break;
        case kF32:
            hipLaunchKernelGGL(k_sweep_gather<float>, dim3(nb), dim3(B), 0, st, (float*)u, tab, s, g);
            break;
        default:
            hipLaunchKernelGGL(k_sweep_gather<bf16s>, dim3(nb), dim3(B), 0, st, (bf16s*)u, tab, s, g);
    }
    return hipGetLastError();
}

// ------------------------------------------------------------- conversions --

template <class T>
__global__ void k_to_f64(const T* __restrict__ src, double* __restrict__ dst, long long n) {
    const long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) dst[i] = (double)ld(src + i);
}

template <class T>
__global__ void k_from_f64(const double* __restrict__ src, T* __restrict__ dst, long long n) {
    const long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) st(dst + i, src[i]);
}

hipError_t launch_to_f64(int prec, const void* src, double* dst, long long n, hipStream_t s) {
    const unsigned nb = (unsigned)((n + 255) / 256);
    if (prec == kF64)
        hipLaunchKernelGGL(k_to_f64<double>, dim3(nb), dim3(256), 0, s, (const double*)src, dst, n);
    else if (prec == kF32)
        hipLaunchKernelGGL(k_to_f64<float>, dim3(nb), dim3(256), 0, s, (const float*)src, dst, n);
    else
        hipLaunchKernelGGL(k_to_f64<bf16s>, dim3(nb), dim3(256), 0, s, (const bf16s*)src, dst, n);
    return hipGetLastError();
}

hipError_t launch_from_f64(int prec, const double* src, void* dst, long long n, hipStream_t s) {
    const unsigned nb = (unsigned)((n + 255) / 256);
    if (prec == kF64)
        hipLaunchKernelGGL(k_from_f64<double>, dim3(nb), dim3(256), 0, s, src, (double*)dst, n);
    else if (prec == kF32)
        hipLaunchKernelGGL(k_from_f64<float>, dim3(nb), dim3(256), 0, s, src, (float*)dst, n);
    else
        hipLaunchKernelGGL(k_from_f64<bf16s>, dim3(nb), dim3(256), 0, s, src, (bf16s*)dst, n);
    return hipGetLastError();
}

__global__ void k_fill_zero(uint32_t* p, long long n) {
    const long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) p[i] = 0u;
}

hipError_t launch_fill_zero(void* p, long long bytes, hipStream_t s) {
    // A fill kernel rather than a memset node: safe under graph capture.
    const long long n = bytes / 4;
    if (n > 0)
        hipLaunchKernelGGL(k_fill_zero, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, s,
                           (uint32_t*)p, n);
    return hipGetLastError();
}

// -------------------------------------------------------------- reductions --
// Fixed-shape two-pass reductions (deterministic order).

template <class T>
__global__ void k_sum_partial(const T* __restrict__ p, long long n, double* __restrict__ part) {
    __shared__ double sh[256];
    double s = 0.0;
    for (long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x; i < n;
         i += (long long)gridDim.x * blockDim.x)
        s += (double)ld(p + i);
    sh[threadIdx.x] = s;
    __syncthreads();
    for (int k = 128; k > 0; k >>= 1) {
        if ((int)threadIdx.x < k) sh[threadIdx.x] += sh[threadIdx.x + k];
        __syncthreads();
    }
    if (threadIdx.x == 0) part[blockIdx.x] = sh[0];
}

__global__ void k_sum_final(const double* __restrict__ part, int npart, double* __restrict__ out) {
    __shared__ double sh[256];
    double s = 0.0;
    for (int i = threadIdx.x; i < npart; i += blockDim.x) s += part[i];
    sh[threadIdx.x] = s;
    __syncthreads();
    for (int k = 128; k > 0; k >>= 1) {
        if ((int)threadIdx.x < k) sh[threadIdx.x] += sh[threadIdx.x + k];
        __syncthreads();
    }
    if (threadIdx.x == 0) *out = sh[0];
}

hipError_t launch_sum(int prec, const void* plane, long long n, double* part, int npart,
                      double* out, hipStream_t s) {
    if (prec == kF64)
        hipLaunchKernelGGL(k_sum_partial<double>, dim3(npart), dim3(256), 0, s, (const double*)plane, n, part);
    else if (prec == kF32)
        hipLaunchKernelGGL(k_sum_partial<float>, dim3(npart), dim3(256), 0, s, (const float*)plane, n, part);
    else
        hipLaunchKernelGGL(k_sum_partial<bf16s>, dim3(npart), dim3(256), 0, s, (const bf16s*)plane, n, part);
    hipLaunchKernelGGL(k_sum_final, dim3(1), dim3(256), 0, s, part, npart, out);
    return hipGetLastError();
}

template <class T>
__global__ void k_check_partial(const T* __restrict__ u, int nplanes, GridDesc g,
                                double* __restrict__ pmax, unsigned long long* __restrict__ pcnt) {
    __shared__ double shm[256];
    __shared__ unsigned long long shc[256];
    double m = 0.0;
    unsigned long long k = 0;
    const long long total = (long long)nplanes * g.ncell;
    for (long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x; i < total;
         i += (long long)gridDim.x * blockDim.x) {
        const long long pl = i / g.ncell, c = i - pl * g.ncell;
        const double v = (double)ld(u + pl * g.pstride + c);
        if (!isfinite(v))
            ++k;
        else
            m = fmax(m, fabs(v));
    }
    shm[threadIdx.x] = m;
    shc[threadIdx.x] = k;
    __syncthreads();
    for (int s = 128; s > 0; s >>= 1) {
        if ((int)threadIdx.x < s) {
            shm[threadIdx.x] = fmax(shm[threadIdx.x], shm[threadIdx.x + s]);
            shc[threadIdx.x] += shc[threadIdx.x + s];
        }
        __syncthreads();
    }
    if (threadIdx.x == 0) {
        pmax[blockIdx.x] = shm[0];
        pcnt[blockIdx.x] = shc[0];
    }
}

__global__ void k_check_final(const double* pmax, const unsigned long long* pcnt, int npart,
                              double* out_max, unsigned long long* out_cnt) {
    if (threadIdx.x == 0 && blockIdx.x == 0) {
        double m = 0.0;
        unsigned long long k = 0;
        for (int i = 0; i < npart; ++i) {
            m = fmax(m, pmax[i]);
            k += pcnt[i];
        }
        *out_max = m;
        *out_cnt = k;
    }
}

hipError_t launch_check(int prec, const void* u, int nplanes, GridDesc g, double* pmax,
                        unsigned long long* pcnt, int npart, double* out_max,
                        unsigned long long* out_cnt, hipStream_t s) {
    if (prec == kF64)
        hipLaunchKernelGGL(k_check_partial<double>, dim3(npart), dim3(256), 0, s, (const double*)u, nplanes, g, pmax, pcnt);
    else if (prec == kF32)
        hipLaunchKernelGGL(k_check_partial<float>, dim3(npart), dim3(256), 0, s, (const float*)u, nplanes, g, pmax, pcnt);
    else
        hipLaunchKernelGGL(k_check_partial<bf16s>, dim3(npart), dim3(256), 0, s, (const bf16s*)u, nplanes, g, pmax, pcnt);
    hipLaunchKernelGGL(k_check_final, dim3(1), dim3(64), 0, s, pmax, pcnt, npart, out_max, out_cnt);
    return hipGetLastError();
}

// ----------------------------------------------------------------- adjoint --
// Transpose of the substep u_i' = alpha_i u_i + beta_i r_i (i of parity p),
// r_i = q_i - sum_d sum_j M_d[i,j] D_d u_j.  With cotangent lam:
//   dL/dalpha_i += lam_i u_i,   dL/dbeta_i += lam_i r_i      (per cell)
//   w_i = beta_i lam_i,         lam_i <- alpha_i lam_i       (k_adj_targets)
//   lam_j += sum_d sum_i M_d[j,i] D_d^(j) w_i   (j dual)     (k_adj_duals)
// The last line uses that the transpose of a forward periodic difference is
// minus the backward one: the dual update has exactly the stencil of a
// forward sweep whose targets are the dual moments, reading w as sources.

template <class T>
__global__ void __launch_bounds__(256) k_adj_targets(const T* __restrict__ uold,
                                                     T* __restrict__ lam, T* __restrict__ w,
                                                     double* __restrict__ grad,
                                                     const double* __restrict__ tab, Schedule s,
                                                     GridDesc g) {
    using A = typename Acc<T>::type;
    const long long c = (long long)blockIdx.x * blockDim.x + threadIdx.x;
    if (c >= g.ncell) return;
    const Nbr n = neighbours(c, g);
    int cur = -1;
    double ga = 0.0, gb = 0.0;
    for (int t = 0; t < s.nrows; ++t) {
        const SweepRow R = s.rows[t];
        const int set = R.tab >> 1;  // grid order, or 8 for moment 0
        if (set != cur) {
            if (cur >= 0) {
                grad[(long long)(2 * cur) * g.ncell + c] += ga;
                grad[(long long)(2 * cur + 1) * g.ncell + c] += gb;
            }
            cur = set;
            ga = gb = 0.0;
        }
        A acc = 0;
        for (int e = R.begin; e < R.end; ++e) {
            const SweepEnt E = s.ents[e];
            const T* uj = uold + (long long)E.slot * g.pstride;
            acc += (A)E.K * ((A)ld(uj + c + pick(n, E.nb)) - (A)ld(uj + c));
        }
        const double alpha = tab[(long long)R.tab * g.ncell + c];
        const double beta = tab[(long long)(R.tab + 1) * g.ncell + c];
        const double q = (R.tab == kTabMom0) ? tab[(long long)kTabQ * g.ncell + c] : 0.0;
        const long long o = (long long)R.slot * g.pstride + c;
        const double l = (double)ld(lam + o);
        ga += l * (double)ld(uold + o);
        gb += l * (q - (double)acc);
        st(w + o, beta * l);
        st(lam + o, alpha * l);
    }
    if (cur >= 0) {
        grad[(long long)(2 * cur) * g.ncell + c] += ga;
        grad[(long long)(2 * cur + 1) * g.ncell + c] += gb;
    }
}

template <class T>
__global__ void __launch_bounds__(256) k_adj_duals(T* __restrict__ lam, const T* __restrict__ w,
                                                   Schedule s, GridDesc g) {
    using A = typename Acc<T>::type;
    const long long c = (long long)blockIdx.x * blockDim.x + threadIdx.x;
    if (c >= g.ncell) return;
    const Nbr n = neighbours(c, g);
    for (int t = 0; t < s.nrows; ++t) {
        const SweepRow R = s.rows[t];
        A acc = 0;
        for (int e = R.begin; e < R.end; ++e) {
            const SweepEnt E = s.ents[e];
            const T* wj = w + (long long)E.slot * g.pstride;
            acc += (A)E.K * ((A)ld(wj + c + pick(n, E.nb)) - (A)ld(wj + c));
        }
        T* lt = lam + (long long)R.slot * g.pstride + c;
        st(lt, (double)ld(lt) + (double)acc);
    }
}

hipError_t launch_adj_targets(int prec, const void* uold, void* lam, void* w, double* grad,
                              const double* tab, Schedule s, GridDesc g, hipStream_t st) {
    const unsigned nb = (unsigned)((g.ncell + 255) / 256);
    if (prec == kF64)
        hipLaunchKernelGGL(k_adj_targets<double>, dim3(nb), dim3(256), 0, st, (const double*)uold, (double*)lam, (double*)w, grad, tab, s, g);
    else if (prec == kF32)
        hipLaunchKernelGGL(k_adj_targets<float>, dim3(nb), dim3(256), 0, st, (const float*)uold, (float*)lam, (float*)w, grad, tab, s, g);
    else
        hipLaunchKernelGGL(k_adj_targets<bf16s>, dim3(nb), dim3(256), 0, st, (const bf16s*)uold, (bf16s*)lam, (bf16s*)w, grad, tab, s, g);
    return hipGetLastError();
}

hipError_t launch_adj_duals(int prec, void* lam, const void* w, Schedule s, GridDesc g,
                            hipStream_t st) {
    const unsigned nb = (unsigned)((g.ncell + 255) / 256);
    if (prec == kF64)
        hipLaunchKernelGGL(k_adj_duals<double>, dim3(nb), dim3(256), 0, st, (double*)lam, (const double*)w, s, g);
    else if (prec == kF32)
        hipLaunchKernelGGL(k_adj_duals<float>, dim3(nb), dim3(256), 0, st, (float*)lam, (const float*)w, s, g);
    else
        hipLaunchKernelGGL(k_adj_duals<bf16s>, dim3(nb), dim3(256), 0, st, (bf16s*)lam, (const bf16s*)w, s, g);
    return hipGetLastError();
}

// d beta / d c for beta = (1 - exp(-c tau))/c:  -tau^2 F(c tau) with
// F(z) = (1 - (1+z) e^{-z}) / z^2 = sum_k (-1)^k (k+1) z^k / (k+2)!,
// summed as a series for |z| < 1e-2 (truncation below 1e-16 relative).
__device__ __forceinline__ double dbeta_dc(double c, double tau, double alpha, double beta) {
    const double z = c * tau;
    if (fabs(z) < 1e-2) {
        const double F = 0.5 + z * (-1.0 / 3.0 + z * (1.0 / 8.0 + z * (-1.0 / 30.0 + z * (1.0 / 144.0 - z / 840.0))));
        return -tau * tau * F;
    }
    return (tau * alpha - beta) / c;
}

// Chain rule to the cell-centred medium: per set s the coefficient c_s on
// the set's points is the mean of (sigma_a [+ sigma_s]) over 2^k cells
// c + b; its transpose gathers g_s from the cells c - b.
__global__ void k_grad_final(const double* __restrict__ grad, const double* __restrict__ tab,
                             const double* __restrict__ sa, const double* __restrict__ ss,
                             double* __restrict__ dsa, double* __restrict__ dss, GridDesc g,
                             double dt) {
    const long long c = (long long)blockIdx.x * blockDim.x + threadIdx.x;
    if (c >= g.ncell) return;
    double ta = 0.0, ts = 0.0;
    for (int s = 0; s < 9; ++s) {
        const int bits = s < 8 ? c_grid_bits[s] : 0;
        const int ox = bits & 1, oy = (bits >> 1) & 1, oz = (bits >> 2) & 1;
        const double tau = set_tau(s, dt);
        const int row = s < 8 ? 2 * s : kTabMom0;
        double acc = 0.0;
        int cnt = 0;
        for (int bz = 0; bz <= oz; ++bz)
            for (int by = 0; by <= oy; ++by)
                for (int bx = 0; bx <= ox; ++bx) {
                    const long long k = shifted(c, bx, by, bz, true, g);
                    const double a = tab[(long long)row * g.ncell + k];
                    const double b = tab[(long long)(row + 1) * g.ncell + k];
                    const double cc = cbar_at(sa, ss, k, s, g);
                    const double ga = grad[(long long)(2 * s) * g.ncell + k];
                    const double gb = grad[(long long)(2 * s + 1) * g.ncell + k];
                    acc += ga * (-tau * a) + gb * dbeta_dc(cc, tau, a, b);
                    ++cnt;
                }
        acc /= cnt;
        ta += acc;
        if (s < 8) ts += acc;
    }
    if (dsa) dsa[c] = ta;
    if (dss) dss[c] = ts;
}

hipError_t launch_grad_final(const double* grad, const double* tab, const double* sa,
                             const double* ss, double* dsa, double* dss, GridDesc g, double dt,
                             hipStream_t st) {
    const unsigned nb = (unsigned)((g.ncell + 255) / 256);
    hipLaunchKernelGGL(k_grad_final, dim3(nb), dim3(256), 0, st, grad, tab, sa, ss, dsa, dss, g, dt);
    return hipGetLastError();
}

}  // namespace pm
