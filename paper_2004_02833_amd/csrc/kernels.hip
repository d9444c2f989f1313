// HIP kernels of libpm for gfx950 (MI355X).
//
// State layout in HBM: moment-major planes, u[slot][z][y][x] with x fastest;
// slots are grouped by staggered grid (G111, G221, G212, G122 | G211, G121,
// G112, G222) so that each parity is one contiguous range.  A lane owns CPL
// consecutive cells of a row (1 for FP64 and FP32, 2 for BF16), so every
// plane access of a wave is a contiguous segment of 64 CPL cells: 512 B
// (FP64), 256 B (FP32, BF16).  Rows of exactly 64 CPL cells are held by one
// wave each, whose x neighbours then come by lane rotation.
#include <hip/hip_runtime.h>

#include <cmath>
#include <cstdint>
#include <type_traits>

#include "kernels.h"

// Target degrees per pass: registers (hence resident waves) and balanced
// passes against re-reading the source degree that adjacent passes share.
// Measured (GDoF-updates/s, FP64 / FP32):
//   N <= 20: K = 2 (P7 at 64^3-160^3: +16% / up to +19%; P19: +8% / +5%);
//   larger N: FP64 K = 3 (P39 64^3 whole-row waves held to 4 waves/SIMD:
//   180 vs 178 at K = 2; 160^3: +5%), FP32 K = 2 where waves hold whole
//   rows (7 waves/SIMD; K = 3 at 7 waves within noise) and K = 3 otherwise
//   (160^3: 306 vs 291); BF16 K = 3.  The transposed sweeps run at K = 2.
#ifndef PM_WIN_K64
#define PM_WIN_K64 3
#endif
#ifndef PM_ADJ_K64
#define PM_ADJ_K64 2
#endif
#ifndef PM_ADJ_K32
#define PM_ADJ_K32 2
#endif
#ifndef PM_WIN_KLOW
#define PM_WIN_KLOW 2   // FP64 and FP32 at N <= PM_N_LOW (PM_N_LOW_LONG on rows > 64)
#endif
#ifndef PM_N_LOW
#define PM_N_LOW 20
#endif
// on rows longer than 64 cells: P19, FP32 500^3 odd + even sweep 149.9 vs
// 160.7 ms at depth 3 / 2, FP64 128^3 5.26 vs 5.41 ms, 160^3 10.34 vs 10.67;
// but P7 and P3 lose 2-24% at depth 3 (P19 FP32 128^3: +4.9%)
#ifndef PM_N_LOW_LONG
#define PM_N_LOW_LONG 15
#endif
#ifndef PM_WIN_K32
#define PM_WIN_K32 2
#endif
#ifndef PM_WIN_K32R
#define PM_WIN_K32R 3
#endif
// BF16 (all orders): P39 64^3 odd + even sweep 0.717 vs 0.832 ms at depth
// 2 / 3, 160^3 10.41 vs 10.51, P19 500^3 105.4 vs 106.0
// anisotropic FP64 (P39 64^3 odd + even sweep 2.242 vs 2.359 ms at depth 2 / 3)
#ifndef PM_WIN_K64A
#define PM_WIN_K64A 2
#endif
#ifndef PM_WIN_K16
#define PM_WIN_K16 2
#endif
#ifndef PM_WIN_K64R
#define PM_WIN_K64R 3   // FP64 where waves do not hold whole rows (P39 160^3: 20.28 vs 20.88 ms at K = 2)
#endif

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

// Two float values rounded to nearest even into bfloat16, the first in the
// low half: one packed hardware conversion (v_cvt_pk_bf16_f32).  For every
// non-NaN input it gives the bits of rounding the float's bit pattern by
// hand (add 0x7fff plus the kept lowest bit, keep the high half), checked
// over all 2^32 inputs; a NaN stays a NaN.
typedef __bf16 bf16x2_t __attribute__((ext_vector_type(2)));
typedef float f32x2_t __attribute__((ext_vector_type(2)));
__device__ __forceinline__ uint32_t bf_pack2(float a, float b) {
    const f32x2_t v = {a, b};
    return __builtin_bit_cast(uint32_t, __builtin_convertvector(v, bf16x2_t));
}

// Round-to-nearest-even conversions from the float64 update (bfloat16: via
// float, as the FP32 form stores it, then to bfloat16).
__device__ __forceinline__ void st(double* p, double v) { *p = v; }
__device__ __forceinline__ void st(float* p, double v) { *p = (float)v; }
__device__ __forceinline__ void st(bf16s* p, double v) {
    p->b = (uint16_t)(bf_pack2((float)v, 0.0f) & 0xffffu);
}

// Streaming (non-temporal) access for values that are read once and written
// once per sweep (the target moments): keeps L2 for the source rows that are
// re-read as neighbours by other waves.
__device__ __forceinline__ double ld_nt(const double* p) { return __builtin_nontemporal_load(p); }
__device__ __forceinline__ float ld_nt(const float* p) { return __builtin_nontemporal_load(p); }
__device__ __forceinline__ float ld_nt(const bf16s* p) {
    return __uint_as_float((uint32_t)__builtin_nontemporal_load(&p->b) << 16);
}
__device__ __forceinline__ void st_nt(double* p, double v) { __builtin_nontemporal_store(v, p); }
__device__ __forceinline__ void st_nt(float* p, double v) { __builtin_nontemporal_store((float)v, p); }
__device__ __forceinline__ void st_nt(bf16s* p, double v) {
    bf16s t;
    st(&t, v);
    __builtin_nontemporal_store(t.b, &p->b);
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

// d beta / d c for beta = (1 - exp(-c tau))/c:  -tau^2 F(c tau) with
// F(z) = (1 - (1+z) e^{-z}) / z^2 = sum_k (-1)^k (k+1) z^k / (k+2)!,
// summed as a series for |z| < 1e-2 (truncation below 1e-16 relative).
__device__ __forceinline__ double dbeta_series(double z, double tau) {
    const double F = 0.5 + z * (-1.0 / 3.0 + z * (1.0 / 8.0 + z * (-1.0 / 30.0 + z * (1.0 / 144.0 - z / 840.0))));
    return -tau * tau * F;
}

__device__ __forceinline__ double dbeta_dc(double c, double tau, double alpha, double beta) {
    const double z = c * tau;
    if (fabs(z) < 1e-2) return dbeta_series(z, tau);
    return (tau * alpha - beta) / c;
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
    for (int f = 0; f < 4; ++f) {
        double a, b;
        decay(cbar_at(sa, ss, c, 4 + f, g), dt, a, b);
        tab[(long long)(kTabOddFull + 2 * f) * g.ncell + c] = a;
        tab[(long long)(kTabOddFull + 2 * f + 1) * g.ncell + c] = b;
    }
}

// Anisotropic scattering: the coefficient of degree l is
// c_l = sigma_a + (1 - g_l) sigma_s, so every grid keeps the means of
// sigma_a and of sigma_s over the cells sharing its point (rows 2s, 2s + 1);
// the sweeps form c_l and its decay factors per degree.  Row 18 holds q.
__device__ __forceinline__ void means_at(const double* __restrict__ sa,
                                         const double* __restrict__ ss, long long c, int s,
                                         const GridDesc& g, double& ma, double& ms) {
    const int bits = c_grid_bits[s];
    const int ox = bits & 1, oy = (bits >> 1) & 1, oz = (bits >> 2) & 1;
    double a = 0.0, b = 0.0;
    int cnt = 0;
    for (int bz = 0; bz <= oz; ++bz)
        for (int by = 0; by <= oy; ++by)
            for (int bx = 0; bx <= ox; ++bx) {
                const long long k = shifted(c, bx, by, bz, false, g);
                a += sa[k];
                b += ss[k];
                ++cnt;
            }
    ma = a / cnt;
    ms = b / cnt;
}

__global__ void k_tables_aniso(const double* __restrict__ sa, const double* __restrict__ ss,
                               const double* __restrict__ q, double* __restrict__ tab,
                               GridDesc g) {
    const long long c = (long long)blockIdx.x * blockDim.x + threadIdx.x;
    if (c >= g.ncell) return;
    for (int s = 0; s < 8; ++s) {
        double ma, ms;
        means_at(sa, ss, c, s, g, ma, ms);
        tab[(long long)(2 * s) * g.ncell + c] = ma;
        tab[(long long)(2 * s + 1) * g.ncell + c] = ms;
    }
    tab[(long long)kTabQ * g.ncell + c] = q ? q[c] : 0.0;
}

// Float copy of the tables for the FP32 update of float and bfloat16
// storage: every alpha row holds gamma = 1 - alpha instead (the update is
// u - gamma u + beta (q - S)), so that rounding the factor to float moves
// the per-step decay by a relative 2^-24 of gamma, not of alpha: no
// systematic drift of order steps * 2^-24 over a run.
__global__ void k_tables_f32(const double* __restrict__ tab, float* __restrict__ tabf,
                             long long n) {
    const long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= (long long)kTabRows * n) return;
    const int row = (int)(i / n);
    const bool alpha = (row < kTabQ && (row & 1) == 0) || (row > kTabQ && ((row - kTabOddFull) & 1) == 0);
    const double v = tab[i];
    tabf[i] = (float)(alpha ? 1.0 - v : v);
}

hipError_t launch_tables_f32(const double* tab, float* tabf, long long n, hipStream_t st) {
    const long long tot = (long long)kTabRows * n;
    hipLaunchKernelGGL(k_tables_f32, dim3((unsigned)((tot + 255) / 256)), dim3(256), 0, st, tab,
                       tabf, n);
    return hipGetLastError();
}

hipError_t launch_tables(const double* sa, const double* ss, const double* q, double* tab,
                         GridDesc g, double dt, bool aniso, hipStream_t st) {
    const int B = 256;
    const long long nb = (g.ncell + B - 1) / B;
    if (aniso)
        hipLaunchKernelGGL(k_tables_aniso, dim3((unsigned)nb), dim3(B), 0, st, sa, ss, q, tab, g);
    else
        hipLaunchKernelGGL(k_tables, dim3((unsigned)nb), dim3(B), 0, st, sa, ss, q, tab, g, dt);
    return hipGetLastError();
}

// ---- several consecutive x-cells per lane --------------------------------
// A lane owns CPL consecutive cells of a row; its plane accesses are vector
// loads/stores of CPL elements (8 to 16 bytes), so a wave moves 512 B to 1 KB
// per instruction whatever the storage type.
template <class T, int CPL> struct Pack;
template <> struct Pack<double, 1> { using V = double; using S1 = double; };
template <> struct Pack<double, 2> { using V = double __attribute__((ext_vector_type(2))); using S1 = double; };
template <> struct Pack<float, 1> { using V = float; using S1 = float; };
template <> struct Pack<float, 2> { using V = float __attribute__((ext_vector_type(2))); using S1 = float; };
template <> struct Pack<float, 4> { using V = float __attribute__((ext_vector_type(4))); using S1 = float; };
template <> struct Pack<bf16s, 1> { using V = uint16_t; using S1 = uint16_t; };
template <> struct Pack<bf16s, 2> { using V = uint32_t; using S1 = uint16_t; };
template <> struct Pack<bf16s, 4> { using V = uint32_t __attribute__((ext_vector_type(2))); using S1 = uint16_t; };

__device__ __forceinline__ float bf_lo(uint32_t w) { return __uint_as_float(w << 16); }
__device__ __forceinline__ float bf_hi(uint32_t w) { return __uint_as_float(w & 0xffff0000u); }
__device__ __forceinline__ uint32_t bf_bits(double v) {
    bf16s t;
    st(&t, v);
    return t.b;
}

template <class T, int CPL, class A>
__device__ __forceinline__ void unpack(typename Pack<T, CPL>::V v, A (&o)[CPL]) {
    if constexpr (std::is_same<T, bf16s>::value) {
        if constexpr (CPL == 1) {
            o[0] = __uint_as_float((uint32_t)v << 16);
        } else if constexpr (CPL == 2) {
            o[0] = bf_lo(v);
            o[1] = bf_hi(v);
        } else {
            o[0] = bf_lo(v.x);
            o[1] = bf_hi(v.x);
            o[2] = bf_lo(v.y);
            o[3] = bf_hi(v.y);
        }
    } else if constexpr (CPL == 1) {
        o[0] = v;
    } else {
#pragma unroll
        for (int k = 0; k < CPL; ++k) o[k] = v[k];
    }
}

template <class T, int CPL>
__device__ __forceinline__ typename Pack<T, CPL>::V pack(const double (&v)[CPL]) {
    using V = typename Pack<T, CPL>::V;
    V r;
    if constexpr (std::is_same<T, bf16s>::value) {
        if constexpr (CPL == 1) {
            r = (uint16_t)bf_bits(v[0]);
        } else if constexpr (CPL == 2) {
            r = bf_pack2((float)v[0], (float)v[1]);
        } else {
            r.x = bf_pack2((float)v[0], (float)v[1]);
            r.y = bf_pack2((float)v[2], (float)v[3]);
        }
    } else if constexpr (CPL == 1) {
        r = (T)v[0];
    } else {
#pragma unroll
        for (int k = 0; k < CPL; ++k) r[k] = (T)v[k];
    }
    return r;
}

// float or bfloat16 storage from float values (the FP32 update)
template <class T, int CPL>
__device__ __forceinline__ typename Pack<T, CPL>::V pack_f(const float (&v)[CPL]) {
    static_assert(!std::is_same<T, double>::value, "float update only for float and bfloat16 storage");
    typename Pack<T, CPL>::V r;
    if constexpr (std::is_same<T, float>::value) {
        if constexpr (CPL == 1) {
            r = v[0];
        } else {
#pragma unroll
            for (int k = 0; k < CPL; ++k) r[k] = v[k];
        }
    } else if constexpr (CPL == 1) {
        r = (uint16_t)(bf_pack2(v[0], 0.0f) & 0xffffu);
    } else if constexpr (CPL == 2) {
        r = bf_pack2(v[0], v[1]);
    } else {
        r.x = bf_pack2(v[0], v[1]);
        r.y = bf_pack2(v[2], v[3]);
    }
    return r;
}

template <class T> __device__ __forceinline__ float s1_val(uint16_t b) { return __uint_as_float((uint32_t)b << 16); }
template <class T> __device__ __forceinline__ T s1_val(T x) { return x; }

// Raw values of one source for one lane: its CPL centre cells, the CPL cells
// of the one-sided y and z neighbour rows, and the one x neighbour outside
// the lane's own cells.
template <class T, int CPL>
struct Raw {
    typename Pack<T, CPL>::V c, y, z;
    typename Pack<T, CPL>::S1 xe;
};

struct LaneNbr {
    long long c0;       // first cell of the lane
    int xep, xem;       // offset of the outside x neighbour: forward, backward
    int yp, ym, zp, zm; // row offsets of the y / z neighbours: forward, backward
};

// How a sweep gets the x neighbour outside a lane's own cells:
//   kXLoad   loaded by every lane (any tiling);
//   kXRow    whole-row waves (64 CPL cells = nx): by lane rotation, the
//            periodic wrap included.
enum XMode { kXLoad = 0, kXRow = 1 };

// Wavefront rotations by one lane (DPP wave_rol:1 / wave_ror:1): lane i
// receives the value of lane i + 1 (next) or i - 1 (prev), modulo 64.
// Every lane of the wave must be active; every lane then reads a valid lane,
// so no old value has to be supplied (no register to clear first).
__device__ __forceinline__ uint32_t rot_next(uint32_t v) {
    return (uint32_t)__builtin_amdgcn_mov_dpp((int)v, 0x134, 0xf, 0xf, false);
}
__device__ __forceinline__ uint32_t rot_prev(uint32_t v) {
    return (uint32_t)__builtin_amdgcn_mov_dpp((int)v, 0x13C, 0xf, 0xf, false);
}
template <bool NEXT> __device__ __forceinline__ double rot(double v) {
    const uint32_t lo = (uint32_t)__double2loint(v), hi = (uint32_t)__double2hiint(v);
    return __hiloint2double((int)(NEXT ? rot_next(hi) : rot_prev(hi)),
                            (int)(NEXT ? rot_next(lo) : rot_prev(lo)));
}
template <bool NEXT> __device__ __forceinline__ float rot(float v) {
    return __uint_as_float(NEXT ? rot_next(__float_as_uint(v)) : rot_prev(__float_as_uint(v)));
}
template <bool NEXT> __device__ __forceinline__ uint16_t rot(uint16_t v) {
    return (uint16_t)(NEXT ? rot_next(v) : rot_prev(v));
}

// kXRow: every wave holds one whole row (64 lanes x CPL cells = nx), so the
// x neighbour outside a lane's cells, periodic wrap included, is held by the
// next or previous lane and comes by a rotation instead of a load.
template <class T, int CPL, int XM>
__device__ __forceinline__ void win_fetch(Raw<T, CPL>& r, const T* __restrict__ u, int2 d,
                                          const LaneNbr& nb, long long ps) {
    using V = typename Pack<T, CPL>::V;
    using S1 = typename Pack<T, CPL>::S1;
    if (d.x >= 0) {
        const T* p = u + (long long)d.x * ps + nb.c0;
        r.c = *(const V*)p;
        r.y = *(const V*)(p + ((d.y & 2) ? nb.ym : nb.yp));
        r.z = *(const V*)(p + ((d.y & 4) ? nb.zm : nb.zp));
        if constexpr (XM == kXLoad) r.xe = *(const S1*)(p + ((d.y & 1) ? nb.xem : nb.xep));
    } else {
        r.c = V{};
        r.y = V{};
        r.z = V{};
        r.xe = S1{};
    }
}

// Work decomposition: (tile of cells) x (pass of K target degrees); passes
// are independent (disjoint targets, read-only sources).  When rows split
// into segments of SW cells (SW = 64, 32 or 16 lanes of CPL cells), a wave
// covers one segment of 64 * CPL / SW consecutive rows and the waves of a
// workgroup are stacked along z, so that most one-sided y/z neighbour rows
// are loaded by the same or a sibling wave; otherwise a tile is TPB * CPL
// consecutive cells.  Workgroups are dispatched round-robin over the 8 XCDs
// (id mod 8), so the id is remapped to give every XCD a contiguous range of
// tiles (x segment fastest, then y, then z): neighbour tiles then run at
// about the same time on the same XCD and share its L2.  Within an XCD the
// most expensive passes (highest degrees) go first.  (Interleaving the
// passes of a tile instead was measured slower.)
constexpr int kXcds = 8;

struct TileMap {
    int sw;        // segment width in cells; 0 for linear tiles; -1 for chunk
                   // tiles (nseg = 1, nty = chunks of 64 cells per x-y plane)
    int nseg;      // segments per row
    int nty, ntz;  // tiles per direction
    int pg;        // adjacent passes dispatched together (1: pass-major)
    int gy, gz;    // tile blocks of gy y-tiles x gz z-tiles (gz = 0: none)
};

// Tile order within the contiguous range of an XCD.  With m.gz > 0 the
// tiles go in blocks of m.gy y-tiles x m.gz z-tiles (segments fastest, then
// y, then z inside a block; blocks by y within a z-group), so the
// workgroups resident at one time cover a compact (y, z) block and more of
// their one-sided neighbour rows are rows a resident sibling reads;
// otherwise segments fastest, then y, then z over the whole grid.
__device__ __forceinline__ long long tile_order(const TileMap& m, long long t) {
    if (m.gz <= 0 || m.sw == 0) return t;
    const long long A = (long long)m.nseg * m.nty;
    const long long zg = t / (A * m.gz);
    long long r = t - zg * A * m.gz;
    const int gz = min(m.gz, m.ntz - (int)zg * m.gz);
    const long long B = (long long)m.nseg * m.gy * gz;
    const long long yb = r / B;
    r -= yb * B;
    const int gy = min(m.gy, m.nty - (int)yb * m.gy);
    const long long seg = r % m.nseg;
    r /= m.nseg;
    const long long ty = yb * m.gy + r % gy;
    const long long tz = zg * m.gz + r / gy;
    return seg + m.nseg * (ty + (long long)m.nty * tz);
}

// Workgroup id -> (tile, pass); false for an id past the grid.  Workgroups
// are dispatched round-robin over the XCDs (id mod 8); each XCD gets a
// contiguous range of per_xcd tiles.  m.pg = 1: pass-major (every tile of
// the heaviest pass first); m.pg = G > 1: G adjacent passes of a tile are
// dispatched together, so the source degree two adjacent passes share is
// read by both at about the same time.
__device__ __forceinline__ bool block_work(const TileMap& m, int npass, int per_xcd,
                                           long long ntile, long long& tile, int& pass) {
    const int xcd = blockIdx.x % kXcds;
    const int j = blockIdx.x / kXcds;
    int ti;
    if (m.pg <= 1) {
        ti = j % per_xcd;
        pass = npass - 1 - j / per_xcd;
    } else {
        const int q = j / (per_xcd * m.pg);
        const int r = j - q * per_xcd * m.pg;
        const int gq = min(m.pg, npass - q * m.pg);
        ti = r / gq;
        pass = npass - 1 - q * m.pg - r % gq;
    }
    const long long t = (long long)xcd * per_xcd + ti;
    if (pass < 0 || t >= ntile) return false;
    tile = tile_order(m, t);
    return true;
}

template <int TPB, int CPL>
__device__ __forceinline__ long long tile_cell(const TileMap& m, long long tile, int tid,
                                               const GridDesc& g, bool& live) {
    if (m.sw == 0) {
        const long long c = (tile * TPB + tid) * CPL;
        live = c < g.ncell;
        return c;
    }
    if (m.sw < 0) {
        // chunk tiles: chunk k of 64 CPL cells of an x-y plane, waves
        // stacked in z; a wave past the grid takes the last plane and lanes
        // past the plane's last cell take its last CPL cells (valid
        // addresses, not stored; nx is a multiple of CPL)
        const long long nxy = (long long)g.nx * g.ny;
        const long long k = tile % m.nty;
        const int zt = (int)(tile / m.nty);
        int z = zt * (TPB / 64) + (tid >> 6);
        long long p = (k * 64 + (tid & 63)) * CPL;
        live = z < g.nz && p < nxy;
        if (z >= g.nz) z = g.nz - 1;
        if (p >= nxy) p = nxy - CPL;
        return (long long)z * nxy + p;
    }
    const int ls = m.sw / CPL;  // lanes per segment row
    const long long xs = tile % m.nseg;
    const long long r = tile / m.nseg;
    const int yt = (int)(r % m.nty);
    const int zt = (int)(r / m.nty);
    const int lane = tid & 63, w = tid >> 6;
    const int x = (int)xs * m.sw + (lane % ls) * CPL;
    const int y = yt * (64 / ls) + lane / ls;
    const int z = zt * (TPB / 64) + w;
    live = y < g.ny && z < g.nz;
    return (long long)x + (long long)g.nx * ((long long)y + (long long)g.ny * z);
}

// Finalisation modes of the window sweep:
//   kFwd     substep of eq. (5): u_i <- alpha u_i + beta (q_i - S_i)
//   kAdjTgt  transpose, target side: with lam_i the cotangent of the updated
//            u_i and S_i recomputed from the old state (its dual half at
//            so.src, its target half at so.aux), add
//            lam_i u_i and lam_i (q_i - S_i) to the gradients of alpha and
//            beta of the target's coefficient set, write w_i = beta lam_i
//            and lam_i <- alpha lam_i
//   kAdjDual transpose, dual side: lam_j <- lam_j + S_j with the sources
//            read from w (the transpose of a forward difference is minus the
//            backward one, so this is a forward-shaped stencil over w)
enum SweepMode { kFwd = 0, kAdjTgt = 1, kAdjDual = 2 };

// Resident waves per SIMD asked of the compiler for the whole-row forward
// sweeps (register budget 512 / waves, checked free of spills); 1 leaves the
// choice to it.
#ifndef PM_WPE64
#define PM_WPE64 4
#endif
#ifndef PM_WPE32
#define PM_WPE32 1
#endif
#ifndef PM_WPE16
#define PM_WPE16 1
#endif
template <class T> struct MinWaves { static constexpr int v = PM_WPE16; };
template <> struct MinWaves<double> { static constexpr int v = PM_WPE64; };
template <> struct MinWaves<float> { static constexpr int v = PM_WPE32; };
// and for the FP64 transposed sweeps (target side, dual side)
#ifndef PM_WPE64_ADJ
#define PM_WPE64_ADJ 4
#endif
#ifndef PM_WPE64_DUAL
#define PM_WPE64_DUAL 4
#endif
// Unused rows added to the LDS table array (a cap on resident workgroups
// for tuning; 0 in use).
#ifndef PM_TL_PAD_ROWS
#define PM_TL_PAD_ROWS 0
#endif
// Dispatch of chunk tiles: groups of adjacent passes and tile blocks
// (chunks x z-tiles; see tile_order and block_work).
#ifndef PM_CHUNK_PASS_GROUP
#define PM_CHUNK_PASS_GROUP 3
#endif
#ifndef PM_CHUNK_GY
#define PM_CHUNK_GY 32
#endif
#ifndef PM_CHUNK_GZ
#define PM_CHUNK_GZ 4
#endif
// Chunk tiles (1): rows of nx > 64 cells whose x-y planes hold whole waves
// are tiled by chunks of 64 consecutive cells of a plane (rows cross chunk
// boundaries; x neighbours loaded), so every plane access of a wave is one
// contiguous 64-cell piece; 0 keeps 16- or 32-lane row segments there.
// PM_CHUNK_RAGGED (1) uses them also where a plane ends inside a chunk
// (its last chunk is partly empty) instead of linear tiles: P19 at 500^3,
// FP32 sweep 80.2 vs 87.5 ms.
#ifndef PM_CHUNK_TILES
#define PM_CHUNK_TILES 1
#endif
#ifndef PM_CHUNK_RAGGED
#define PM_CHUNK_RAGGED 1
#endif
// chunk tiles also for two cells per lane (BF16: chunks of 128 cells)
#ifndef PM_CHUNK_TILES2
#define PM_CHUNK_TILES2 1
#endif
// and at depth 2 (FP64: 5 waves spill 56 B, so the compiler's choice; BF16
// two cells per lane: 6 waves at 80 VGPRs, odd + even sweep P39 64^3 0.694
// vs 0.733 ms, 160^3 10.22 vs 10.62, P19 500^3 95.3 vs 108.6; 7 spill)
#ifndef PM_WPE64N2
#define PM_WPE64N2 1
#endif
#ifndef PM_WPE16N2
#define PM_WPE16N2 6
#endif
// resident waves asked for the FP32 forward sweeps with loaded x neighbours
// (one cell per lane): 6 keeps depth 3 at 80 VGPRs without spills (5
// otherwise); P39 160^3 odd + even 18.07 vs 18.16 ms, P19 500^3 147.7 vs
// 149.1, P7 160^3 0.866 vs 0.901
#ifndef PM_WPE32N
#define PM_WPE32N 6
#endif
// resident waves asked for the FP64 forward sweeps with loaded x neighbours
#ifndef PM_WPE64N
#define PM_WPE64N 1
#endif
template <class T, int K, int MODE, bool ANI, int XM, int CPL>
constexpr int min_waves() {
    if (MODE == kFwd && XM == kXLoad && !ANI && std::is_same<T, double>::value && K == 2) return PM_WPE64N2;
    if (MODE == kFwd && XM == kXLoad && !ANI && std::is_same<T, bf16s>::value && K == 2) return PM_WPE16N2;
    if (MODE == kFwd && XM == kXLoad && !ANI && std::is_same<T, double>::value) return PM_WPE64N;
    if (MODE == kFwd && XM == kXLoad && !ANI && std::is_same<T, float>::value && CPL == 1) return PM_WPE32N;
    if (MODE == kFwd) return XM == kXRow && !ANI ? MinWaves<T>::v : 1;
    if (!std::is_same<T, double>::value || ANI) return 1;
    return MODE == kAdjTgt ? PM_WPE64_ADJ : PM_WPE64_DUAL;
}

// One kernel for the forward substep and both halves of its transpose.
// ANI (anisotropic scattering): the table rows of the four target grids hold
// the means of sigma_a and sigma_s; the decay factors of every (target
// degree, grid) pair of the pass are formed once per cell from
// c_l = mean sigma_a + (1 - g_l) mean sigma_s with the per-degree moments gl
// and the substep length tau, and kept in LDS.  XM: how the x neighbours
// come (XMode), in every mode: the push phase is the same forward-shaped
// stencil for the transposed sweeps.
template <class T, int K, int TPB, int CPL, int MODE, bool ANI, int XM>
__global__ void __launch_bounds__(TPB, (min_waves<T, K, MODE, ANI, XM, CPL>()))
k_sweep_win(T* __restrict__ pool, StateOffs so, double* __restrict__ gp,
            const double* __restrict__ tab, const float* __restrict__ tabf,
            const int2* __restrict__ src, const int2* __restrict__ tgt,
            const typename Acc<T>::type* __restrict__ coef, const double* __restrict__ gl,
            double tau, int rowbase, int N, int parity, int npass, int per_xcd, long long ntile,
            TileMap tm, GridDesc g) {
    static_assert(MODE == kFwd || CPL == 1, "transposed sweeps use one cell per lane");
    static_assert(!(ANI && MODE == kAdjDual), "the dual side reads no decay factors");
    // every plane is addressed from one base: sources (the dual parity),
    // targets read and written (equal offsets for an update in place)
    const T* sv = pool + so.src;
    const T* tin = pool + so.tin;
    T* tout = pool + so.tout;
    using A = typename Acc<T>::type;
    using V = typename Pack<T, CPL>::V;
    long long tile;
    int pass;
    if (!block_work(tm, npass, per_xcd, ntile, tile, pass)) return;
    bool live;
    const long long cl = tile_cell<TPB, CPL>(tm, tile, threadIdx.x, g, live);
    LaneNbr nb;
    {
        // chunk tiles give every wave a valid chunk, also past the grid
        const long long c = (live || tm.sw < 0) ? cl : g.ncell - CPL;
        const Nbr n0 = neighbours(c, g);
        const int x0 = (int)(c % g.nx);
        nb.c0 = c;
        nb.xep = (x0 + CPL == g.nx) ? CPL - g.nx : CPL;
        nb.xem = (x0 == 0) ? g.nx - 1 : -1;
        nb.yp = n0.off[2];
        nb.ym = n0.off[3];
        nb.zp = n0.off[4];
        nb.zm = n0.off[5];
    }
    if constexpr (XM == kXRow) {
        // a wave is one row (or, past the grid, one cell): its y and z
        // neighbour rows are the same for every lane, so the offsets and the
        // choice between them live in scalar registers
        nb.yp = __builtin_amdgcn_readfirstlane(nb.yp);
        nb.ym = __builtin_amdgcn_readfirstlane(nb.ym);
        nb.zp = __builtin_amdgcn_readfirstlane(nb.zp);
        nb.zm = __builtin_amdgcn_readfirstlane(nb.zm);
    }
    if (tm.sw < 0) {
        // chunk tiles: a wave is 64 consecutive cells of one x-y plane, so
        // its z neighbour offsets are wave-uniform
        nb.zp = __builtin_amdgcn_readfirstlane(nb.zp);
        nb.zm = __builtin_amdgcn_readfirstlane(nb.zm);
    }
    const long long ps = g.pstride;
    // decay factors for the lane's cells, kept in LDS instead of registers:
    // isotropic: the four target grids (rows 0..7), moment 0 (8, 9), q (10);
    // ANI: target degree t and grid f in rows 2 (4 t + f), 2 (4 t + f) + 1,
    // q in row 8 K
    constexpr int kRowQ = ANI ? 8 * K : 10;
    // FP32 and BF16 storage: the forward update runs in FP32 from factors
    // rounded to float (gamma = 1 - alpha and beta, computed in FP64): half
    // the LDS and, isotropic, half the table reads (float tables); the
    // transposed sweeps keep FP64 factors
    constexpr bool kF32Update = !std::is_same<T, double>::value && MODE == kFwd;
    using TabT = typename std::conditional<kF32Update, float, double>::type;
    __shared__ TabT tl[kRowQ + 1 + PM_TL_PAD_ROWS][TPB * CPL];
    const int tid = threadIdx.x;
    const int MU1 = N + 3;  // source columns 0..N+1 and an empty column N+2
    const int L0 = parity + 2 * K * pass;
    if (ANI) {
#pragma unroll
        for (int f = 0; f < 4; ++f)
#pragma unroll
            for (int k = 0; k < CPL; ++k) {
                const double ma = tab[(long long)(rowbase + 2 * f) * g.ncell + nb.c0 + k];
                const double ms = tab[(long long)(rowbase + 2 * f + 1) * g.ncell + nb.c0 + k];
#pragma unroll
                for (int t = 0; t < K; ++t) {
                    if (L0 + 2 * t > N) continue;
                    double a, b;
                    decay(ma + (1.0 - gl[L0 + 2 * t]) * ms, tau, a, b);
                    tl[2 * (4 * t + f)][tid * CPL + k] = kF32Update ? 1.0 - a : a;
                    tl[2 * (4 * t + f) + 1][tid * CPL + k] = b;
                }
            }
    } else if (MODE != kAdjDual) {
#pragma unroll
        for (int f = 0; f < 8; ++f)
#pragma unroll
            for (int k = 0; k < CPL; ++k)
                tl[f][tid * CPL + k] = kF32Update ? (TabT)tabf[(long long)(rowbase + f) * g.ncell + nb.c0 + k]
                                                  : (TabT)tab[(long long)(rowbase + f) * g.ncell + nb.c0 + k];
    }
    // kAdjTgt gradient sums: per coefficient set (isotropic), or per grid
    // with respect to the means of sigma_a (ga) and sigma_s (gb) (ANI)
    double ga[5] = {0, 0, 0, 0, 0}, gb[5] = {0, 0, 0, 0, 0};
    // moment 0 (and its source q) is a target of the first even pass only
    if (MODE != kAdjDual && parity == 0 && pass == 0) {
#pragma unroll
        for (int k = 0; k < CPL; ++k) {
            if (!ANI) {
                tl[8][tid * CPL + k] = kF32Update ? (TabT)tabf[(long long)kTabMom0 * g.ncell + nb.c0 + k]
                                                  : (TabT)tab[(long long)kTabMom0 * g.ncell + nb.c0 + k];
                tl[9][tid * CPL + k] = kF32Update ? (TabT)tabf[(long long)(kTabMom0 + 1) * g.ncell + nb.c0 + k]
                                                  : (TabT)tab[(long long)(kTabMom0 + 1) * g.ncell + nb.c0 + k];
            }
            tl[kRowQ][tid * CPL + k] = (kF32Update && !ANI) ? (TabT)tabf[(long long)kTabQ * g.ncell + nb.c0 + k]
                                                            : (TabT)tab[(long long)kTabQ * g.ncell + nb.c0 + k];
        }
    }
    const int mumax = min(N, L0 + 2 * (K - 1));  // largest target |m| in the pass
    const int2* sd = src + (long long)pass * MU1 * (K + 1) * 2;
    const int2* td = tgt + (long long)pass * MU1 * K * 2;
    const A* cf = coef + (long long)pass * MU1 * (K + 1) * 20;

    Raw<T, CPL> R[K + 1][2];  // raw values of the current source column
    // forward sweep: old values of the targets finished in the next column,
    // requested one column ahead (transposed modes read theirs in place)
    typename Pack<T, CPL>::V tpf[K][2];
    if constexpr (MODE == kFwd) {
#pragma unroll
        for (int t = 0; t < K; ++t)
#pragma unroll
            for (int ty = 0; ty < 2; ++ty) {
                const int2 dn = td[t * 2 + ty];
                tpf[t][ty] = dn.x >= 0 ? __builtin_nontemporal_load((const V*)(tin + (long long)dn.x * ps + nb.c0)) : V{};
            }
    }
    A S[3][K][2][CPL];        // partial sums: target columns mu-1, mu, mu+1
#pragma unroll
    for (int b = 0; b <= K; ++b)
#pragma unroll
        for (int ty = 0; ty < 2; ++ty) win_fetch<T, CPL, XM>(R[b][ty], sv, sd[b * 2 + ty], nb, ps);
#pragma unroll
    for (int w = 0; w < 3; ++w)
#pragma unroll
        for (int t = 0; t < K; ++t)
#pragma unroll
            for (int ty = 0; ty < 2; ++ty)
#pragma unroll
                for (int k = 0; k < CPL; ++k) S[w][t][ty][k] = (A)0;

    for (int mu = 0; mu <= mumax + 1; ++mu) {
        const int2* sdc = sd + mu * (K + 1) * 2;
        const int2* sdn = sdc + (K + 1) * 2;
        const A* cfc = cf + (long long)mu * (K + 1) * 20;
        // push every source of column mu, then request its next column
#pragma unroll
        for (int b = 0; b <= K; ++b) {
#pragma unroll
            for (int ty = 0; ty < 2; ++ty) {
                const int2 e = sdc[b * 2 + ty];
                A vc[CPL], vy[CPL], vz[CPL];
                unpack<T, CPL, A>(R[b][ty].c, vc);
                unpack<T, CPL, A>(R[b][ty].y, vy);
                unpack<T, CPL, A>(R[b][ty].z, vz);
                const bool back = e.y & 1;
                A xv;
                if constexpr (XM != kXLoad) {
                    // first cell of the next lane, or last cell of the previous one
                    using S1 = typename Pack<T, CPL>::S1;
                    S1 first, last;
                    if constexpr (CPL == 1) {
                        first = last = (S1)R[b][ty].c;
                    } else if constexpr (std::is_same<T, bf16s>::value) {
                        static_assert(CPL == 2, "bf16 rows by rotation: two cells per lane");
                        first = (S1)(R[b][ty].c & 0xffffu);
                        last = (S1)(R[b][ty].c >> 16);
                    } else {
                        first = R[b][ty].c[0];
                        last = R[b][ty].c[CPL - 1];
                    }
                    // both rotations and a select rather than a branch
                    const S1 from_prev = rot<false>(last), from_next = rot<true>(first);
                    xv = (A)s1_val<T>(back ? from_prev : from_next);
                } else {
                    xv = (A)s1_val<T>(R[b][ty].xe);
                }
                A dx[CPL], dy[CPL], dz[CPL];
#pragma unroll
                for (int k = 0; k < CPL; ++k) {
                    const A xn = back ? (k > 0 ? vc[k > 0 ? k - 1 : 0] : xv)
                                      : (k < CPL - 1 ? vc[k < CPL - 1 ? k + 1 : 0] : xv);
                    dx[k] = xn - vc[k];
                    dy[k] = vy[k] - vc[k];
                    dz[k] = vz[k] - vc[k];
                }
                // Empty asm taking the differences: they are formed here and
                // not sunk into the branch below, past the loads of the next
                // column, where the old source values would stay live beside
                // the new ones (more registers, copies at the loop edge).
#pragma unroll
                for (int k = 0; k < CPL; ++k) asm volatile("" ::"v"(dx[k]), "v"(dy[k]), "v"(dz[k]));
                // the stream ends with an empty column, so the next one can
                // always be requested
                win_fetch<T, CPL, XM>(R[b][ty], sv, sdn[b * 2 + ty], nb, ps);
                if (e.x < 0) continue;
#pragma unroll
                for (int side = 0; side < 2; ++side) {
                    const int t = side == 0 ? b : b - 1;
                    if (t < 0 || t >= K) continue;
                    const A* kk = cfc + ((b * 2 + ty) * 2 + side) * 5;
                    const A k0 = kk[0], k1 = kk[1], k2 = kk[2], k3 = kk[3], k4 = kk[4];
#pragma unroll
                    for (int k = 0; k < CPL; ++k) {
                        S[0][t][ty][k] += k0 * dx[k];
                        S[0][t][1 - ty][k] += k1 * dy[k];
                        S[1][t][ty][k] += k2 * dz[k];
                        S[2][t][ty][k] += k3 * dx[k];
                        S[2][t][1 - ty][k] += k4 * dy[k];
                    }
                }
            }
        }
        // column mu-1 is complete: u <- alpha u + beta (q - sum)
        if (mu >= 1) {
            const int2* tdc = td + (mu - 1) * K * 2;
            typename Pack<T, CPL>::V tcur[K][2];
            if constexpr (MODE == kFwd) {
#pragma unroll
                for (int t = 0; t < K; ++t)
#pragma unroll
                    for (int ty = 0; ty < 2; ++ty) tcur[t][ty] = tpf[t][ty];
                {
                    const int2* tdn = td + mu * K * 2;
#pragma unroll
                    for (int t = 0; t < K; ++t)
#pragma unroll
                        for (int ty = 0; ty < 2; ++ty) {
                            const int2 dn = tdn[t * 2 + ty];
                            tpf[t][ty] = dn.x >= 0 ? __builtin_nontemporal_load(
                                                         (const V*)(tin + (long long)dn.x * ps + nb.c0))
                                                   : V{};
                        }
                }
            }
#pragma unroll
            for (int t = 0; t < K; ++t) {
#pragma unroll
                for (int ty = 0; ty < 2; ++ty) {
                    const int2 d = tdc[t * 2 + ty];
                    if (d.x < 0) continue;
                    // only the degree-0 cos slot can be moment 0 (a test the
                    // compiler drops for every other slot)
                    const bool m0 = t == 0 && ty == 0 && d.y == kTabMom0;
                    // moment 0 (row code kTabMom0) is grid G111, degree 0, under ANI
                    const int ra = ANI ? 2 * (4 * t + ((d.y >> 1) & 3))
                                       : m0 ? 8 : 2 * ((d.y >> 1) & 3);
                    T* ut = tout + (long long)d.x * ps + nb.c0;
                    A old[CPL];
                    if constexpr (MODE == kFwd)
                        unpack<T, CPL, A>(tcur[t][ty], old);
                    else
                        unpack<T, CPL, A>(__builtin_nontemporal_load((const V*)(tin + (long long)d.x * ps + nb.c0)), old);
                    if constexpr (MODE == kFwd && kF32Update) {
                        float nf[CPL];
#pragma unroll
                        for (int k = 0; k < CPL; ++k) {
                            // u - gamma u + beta (q - S)
                            const float q = m0 ? (float)tl[kRowQ][tid * CPL + k] : 0.0f;
                            const float uo = (float)old[k];
                            nf[k] = __builtin_fmaf((float)tl[ra + 1][tid * CPL + k], q - (float)S[0][t][ty][k],
                                                   __builtin_fmaf(-(float)tl[ra][tid * CPL + k], uo, uo));
                        }
                        if (live) __builtin_nontemporal_store(pack_f<T, CPL>(nf), (V*)ut);
                        continue;
                    }
                    double nv[CPL];
                    if constexpr (MODE == kFwd) {
#pragma unroll
                        for (int k = 0; k < CPL; ++k) {
                            const double q = m0 ? tl[kRowQ][tid * CPL + k] : 0.0;
                            nv[k] = tl[ra][tid * CPL + k] * (double)old[k] +
                                    tl[ra + 1][tid * CPL + k] * (q - (double)S[0][t][ty][k]);
                        }
                    } else if constexpr (MODE == kAdjDual) {
                        nv[0] = (double)old[0] + (double)S[0][t][ty][0];
                    } else {
                        // old[0] is lam_i; the old u_i comes from the source state
                        const double lam = (double)old[0];
                        const double uo = (double)ld(pool + so.aux + (long long)d.x * ps + nb.c0);
                        const double q = m0 ? tl[kRowQ][tid] : 0.0;
                        const double r = q - (double)S[0][t][ty][0];
                        if constexpr (ANI) {
                            // dL/dc = lam (u d alpha/dc + r d beta/dc), with c
                            // recovered from the factors: c = (1 - alpha)/beta
                            const double al = tl[ra][tid], be = tl[ra + 1][tid];
                            const double om = 1.0 - al;
                            double db;
                            if (om < 1e-2)
                                db = dbeta_series(tau * om / be, tau);
                            else
                                db = (tau * al - be) * be / om;
                            const double gx = lam * (uo * (-tau * al) + r * db);
                            const double ws = 1.0 - gl[L0 + 2 * t];
                            const int f = (d.y >> 1) & 3;
#pragma unroll
                            for (int f4 = 0; f4 < 4; ++f4)
                                if (f4 == f) {
                                    ga[f4] += gx;
                                    gb[f4] += ws * gx;
                                }
                        } else {
                            const int set = m0 ? 4 : ((d.y >> 1) & 3);
#pragma unroll
                            for (int s5 = 0; s5 < 5; ++s5)
                                if (s5 == set) {
                                    ga[s5] += lam * uo;
                                    gb[s5] += lam * r;
                                }
                        }
                        const double wv[1] = {tl[ra + 1][tid] * lam};
                        if (live) st(pool + so.w + (long long)d.x * ps + nb.c0, wv[0]);
                        nv[0] = tl[ra][tid] * lam;
                    }
                    if (live) __builtin_nontemporal_store(pack<T, CPL>(nv), (V*)ut);
                }
            }
        }
#pragma unroll
        for (int t = 0; t < K; ++t)
#pragma unroll
            for (int ty = 0; ty < 2; ++ty)
#pragma unroll
                for (int k = 0; k < CPL; ++k) {
                    S[0][t][ty][k] = S[1][t][ty][k];
                    S[1][t][ty][k] = S[2][t][ty][k];
                    S[2][t][ty][k] = (A)0;
                }
        // Whole-row waves: one barrier per column keeps the four z-stacked
        // waves of the workgroup on the same column, so the rows a wave reads
        // as z neighbours were just read by its sibling and are still cached
        // (+1.6-2% FP64, +0.5% FP32; flat for loaded x neighbours).  Every
        // wave of a workgroup runs the same pass, so all reach it equally often.
        if constexpr (XM == kXRow) __syncthreads();
    }
    if constexpr (MODE == kAdjTgt) {
        // gradient rows of this pass (2 s for alpha, 2 s + 1 for beta, s the
        // coefficient set: grid order, 8 for moment 0); one workgroup owns
        // every (pass, cell), so the accumulation needs no atomics
        if (live) {
            double* gq = gp + (long long)pass * kGradRows * g.ncell + nb.c0;
            const int gbase = parity ? 4 : 0;
#pragma unroll
            for (int s5 = 0; s5 < 5; ++s5) {
                if (s5 == 4 && (parity != 0 || ANI)) continue;
                const int row = s5 == 4 ? kTabMom0 : 2 * (gbase + s5);
                gq[(long long)row * g.ncell] += ga[s5];
                gq[(long long)(row + 1) * g.ncell] += gb[s5];
            }
        }
    }
}

// Deepest forward pass instantiated for FP64 and FP32 (3, or 4 for tuning).
#ifndef PM_MAX_K
#define PM_MAX_K 3
#endif
static_assert(PM_ADJ_K64 >= 2 && PM_ADJ_K64 <= 3 && PM_ADJ_K32 >= 2 && PM_ADJ_K32 <= 3 &&
                  PM_WIN_K64 >= 2 && PM_WIN_K64 <= PM_MAX_K && PM_WIN_K32 >= 2 &&
                  PM_WIN_K32 <= PM_MAX_K && PM_WIN_K32R >= 2 && PM_WIN_K32R <= PM_MAX_K &&
                  PM_WIN_KLOW >= 2 && PM_WIN_KLOW <= PM_MAX_K && PM_MAX_K <= 4 &&
                  PM_WIN_K64R >= 2 && PM_WIN_K64R <= PM_MAX_K && PM_WIN_K64A >= 2 &&
                  PM_WIN_K64A <= PM_MAX_K,
              "forward FP64 and FP32 sweeps are instantiated for depths 2..PM_MAX_K, "
              "the transposed ones for 2 and 3");

// FP32 forward sweeps of low orders (N <= PM_ROW2_NMAX) on rows of 128
// cells: two cells per lane, so that every wave holds a whole row (x
// neighbours by rotation).  Measured on 128^3, FP32 odd sweep: P7 0.196 vs
// 0.236 ms, P3 0.061 vs 0.070; slower at P19 (1.255 vs 1.202) and P39
// (5.07 vs 4.66), and on chunk tiles (P7 160^3 0.468 vs 0.443).
#ifndef PM_ROW2_NMAX
#define PM_ROW2_NMAX 10
#endif

int win_depth(int prec, int nx, int N, bool aniso) {
    if (prec == kBF16) return PM_WIN_K16;
    // anisotropic FP64: the per-degree factors of K target degrees fill
    // (8K + 1) LDS rows of 2 KB; depth 3 (50 KB) leaves 3 workgroups per CU
    if (prec == kF64 && aniso) return PM_WIN_K64A;
    // rows longer than 64 cells (chunk or segment tiles), except FP32 rows of
    // 128 cells at two cells per lane, take the deeper passes from a lower N
    const bool long_rows = nx > 64 && !(prec == kF32 && nx == 128 && N <= PM_ROW2_NMAX);
    if (N <= (long_rows ? PM_N_LOW_LONG : PM_N_LOW)) return PM_WIN_KLOW;
    if (prec == kF64) return nx == 64 ? PM_WIN_K64 : PM_WIN_K64R;
    return nx == 64 ? PM_WIN_K32 : PM_WIN_K32R;  // FP32: one cell per lane
}
int adj_depth(int prec) { return prec == kF64 ? PM_ADJ_K64 : prec == kF32 ? PM_ADJ_K32 : PM_WIN_K16; }


// Launch shape, measured on P39 64^3.  Cells per lane: 1 for FP64 and FP32
// (2 was slower: more registers per wave), 2 for BF16 (4-byte accesses; +7%).
// Workgroups of 256 / CPL threads keep the LDS decay tables at 22.5 KB
// (11 KB for BF16, which stages them as float);
// 512- and 1024-thread groups (up to 16 row segments stacked in z) were not
// faster in FP64 and slower in FP32.
#ifndef PM_CPL16
#define PM_CPL16 2
#endif

template <class T, int K, int CPL, int MODE, bool ANI>
static void launch_win_t(T* pool, StateOffs so, double* gp, const double* tab, const float* tabf,
                         int rowbase,
                         Aniso an, WinArgs a, GridDesc g, hipStream_t st) {
    using A = typename Acc<T>::type;
    constexpr int TPB = 256 / CPL;
    TileMap tm{0, 1, 1, 1, 1, 0, 0};
    long long ntile = (g.ncell / CPL + TPB - 1) / TPB;
    int sw = 0;
    for (int lanes = 64; lanes >= 16 && !sw; lanes /= 2)
        if (g.nx % (lanes * CPL) == 0) sw = lanes * CPL;
    if (sw) {
        tm.sw = sw;
        tm.nseg = g.nx / sw;
        tm.nty = (g.ny + 64 * CPL / sw - 1) / (64 * CPL / sw);
        tm.ntz = (g.nz + TPB / 64 - 1) / (TPB / 64);
        ntile = (long long)tm.nseg * tm.nty * tm.ntz;
    }
    const int per_xcd = (int)((ntile + kXcds - 1) / kXcds);
    const unsigned nwg = (unsigned)((long long)kXcds * per_xcd * a.npass);
    // one whole row per wave: x neighbours by lane rotation
    if (sw == g.nx && g.nx == 64 * CPL) {
        hipLaunchKernelGGL((k_sweep_win<T, K, TPB, CPL, MODE, ANI, kXRow>), dim3(nwg),
                           dim3(TPB), 0, st, pool, so, gp, tab, tabf, a.src, a.tgt, (const A*)a.coef,
                           an.gl, an.tau, rowbase, a.N, a.parity, a.npass, per_xcd, ntile, tm, g);
        return;
    }
    {
        // rows of nx > 64 cells whose x-y planes hold whole waves: chunk
        // tiles of 64 CPL cells, waves stacked in z
        const long long nxy = (long long)g.nx * g.ny;
        if (PM_CHUNK_TILES && (CPL == 1 || PM_CHUNK_TILES2) && g.nx > 64 && g.nx % CPL == 0 &&
            (nxy % (64 * CPL) == 0 || (PM_CHUNK_RAGGED && sw == 0))) {
            // grouped passes and tile blocks: measured on P39 at 160^3
            // (FP64 -3.6%, FP32 -9.2% sweep time with both); whole-row waves
            // keep pass-major order, where grouping was slower (64^3: +1.4%
            // FP64 with groups of 3)
            TileMap tc{-1, 1, (int)((nxy + 64 * CPL - 1) / (64 * CPL)), (g.nz + TPB / 64 - 1) / (TPB / 64),
                       PM_CHUNK_PASS_GROUP, PM_CHUNK_GY, PM_CHUNK_GZ};
            const long long nt = (long long)tc.nty * tc.ntz;
            const int px = (int)((nt + kXcds - 1) / kXcds);
            const unsigned nw = (unsigned)((long long)kXcds * px * a.npass);
            hipLaunchKernelGGL((k_sweep_win<T, K, TPB, CPL, MODE, ANI, kXLoad>), dim3(nw),
                               dim3(TPB), 0, st, pool, so, gp, tab, tabf, a.src, a.tgt,
                               (const A*)a.coef, an.gl, an.tau, rowbase, a.N, a.parity, a.npass,
                               px, nt, tc, g);
            return;
        }
    }
    hipLaunchKernelGGL((k_sweep_win<T, K, TPB, CPL, MODE, ANI, kXLoad>), dim3(nwg), dim3(TPB),
                       0, st, pool, so, gp, tab, tabf, a.src, a.tgt, (const A*)a.coef, an.gl,
                       an.tau, rowbase, a.N, a.parity, a.npass, per_xcd, ntile, tm, g);
}

template <class T, int K, int CPL>
static void launch_fwd(void* pool, StateOffs so, const double* tab, const float* tabf, int rowbase, Aniso an,
                       WinArgs a, GridDesc g, hipStream_t st) {
    if (an.gl)
        launch_win_t<T, K, CPL, kFwd, true>((T*)pool, so, nullptr, tab, tabf, rowbase, an, a, g, st);
    else
        launch_win_t<T, K, CPL, kFwd, false>((T*)pool, so, nullptr, tab, tabf, rowbase, an, a, g, st);
}

hipError_t launch_sweep_win(int prec, void* pool, StateOffs so, const double* tab, const float* tabf,
                            int rowbase,
                            Aniso an, WinArgs a, GridDesc g, hipStream_t st) {
    if (a.K != win_depth(prec, g.nx, a.N, an.gl != nullptr)) return hipErrorInvalidValue;
    // several cells per lane need whole lane groups within every row
    // FP64 and FP32 sweeps come in depths 2 and 3
    if (prec == kF64) {
        if (a.K == 2)
            launch_fwd<double, 2, 1>(pool, so, tab, tabf, rowbase, an, a, g, st);
#if PM_MAX_K >= 4
        else if (a.K == 4)
            launch_fwd<double, 4, 1>(pool, so, tab, tabf, rowbase, an, a, g, st);
#endif
        else
            launch_fwd<double, 3, 1>(pool, so, tab, tabf, rowbase, an, a, g, st);
    } else if (prec == kF32) {
        if (a.N <= PM_ROW2_NMAX && a.K == 2 && g.nx == 128)
            launch_fwd<float, 2, 2>(pool, so, tab, tabf, rowbase, an, a, g, st);
        else if (a.K == 2)
            launch_fwd<float, 2, 1>(pool, so, tab, tabf, rowbase, an, a, g, st);
#if PM_MAX_K >= 4
        else if (a.K == 4)
            launch_fwd<float, 4, 1>(pool, so, tab, tabf, rowbase, an, a, g, st);
#endif
        else
            launch_fwd<float, 3, 1>(pool, so, tab, tabf, rowbase, an, a, g, st);
    } else {
        if (PM_CPL16 > 1 && g.nx % PM_CPL16 == 0)
            launch_fwd<bf16s, PM_WIN_K16, PM_CPL16>(pool, so, tab, tabf, rowbase, an, a, g, st);
        else
            launch_fwd<bf16s, PM_WIN_K16, 1>(pool, so, tab, tabf, rowbase, an, a, g, st);
    }
    return hipGetLastError();
}

template <class T, int K>
static void launch_adj_t(int side, void* pool, StateOffs so, double* gp, const double* tab,
                         int rowbase, Aniso an, WinArgs a, GridDesc g, hipStream_t st) {
    if (side == 1)
        launch_win_t<T, K, 1, kAdjDual, false>((T*)pool, so, nullptr, tab, nullptr, 0, an, a, g, st);
    else if (an.gl)
        launch_win_t<T, K, 1, kAdjTgt, true>((T*)pool, so, gp, tab, nullptr, rowbase, an, a, g, st);
    else
        launch_win_t<T, K, 1, kAdjTgt, false>((T*)pool, so, gp, tab, nullptr, rowbase, an, a, g, st);
}

hipError_t launch_adj_win(int prec, int side, void* pool, StateOffs so, double* gp,
                          const double* tab, int rowbase, Aniso an, WinArgs a, GridDesc g,
                          hipStream_t st) {
    if (a.K != adj_depth(prec) || prec == kBF16) return hipErrorInvalidValue;
    if (prec == kF64)
        launch_adj_t<double, PM_ADJ_K64>(side, pool, so, gp, tab, rowbase, an, a, g, st);
    else
        launch_adj_t<float, PM_ADJ_K32>(side, pool, so, gp, tab, rowbase, an, a, g, st);
    return hipGetLastError();
}

// Sum of the per-pass gradient rows: grad[row][c] = sum over buffers.
__global__ void k_grad_sum(const double* __restrict__ gp, int nbuf, double* __restrict__ grad,
                           long long n) {
    const long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= (long long)kGradRows * n) return;
    double acc = 0.0;
    for (int b = 0; b < nbuf; ++b) acc += gp[(long long)b * kGradRows * n + i];
    grad[i] = acc;
}

hipError_t launch_grad_sum(const double* gp, int nbuf, double* grad, long long n, hipStream_t st) {
    const long long tot = (long long)kGradRows * n;
    hipLaunchKernelGGL(k_grad_sum, dim3((unsigned)((tot + 255) / 256)), dim3(256), 0, st, gp, nbuf,
                       grad, n);
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

// Largest |u| and count of non-finite values over the first nplanes planes.
// Planes are walked one after another (no division per element); within a
// plane every thread reads 16 bytes at a time (planes start 64-element
// aligned), the last ncell mod VEC cells one by one.
template <class T>
__device__ __forceinline__ void check_vals(const uint4& w, double& m, unsigned long long& k) {
    constexpr int VEC = 16 / sizeof(T);
    double v[VEC];
    if constexpr (std::is_same<T, double>::value) {
        v[0] = __hiloint2double((int)w.y, (int)w.x);
        v[1] = __hiloint2double((int)w.w, (int)w.z);
    } else if constexpr (std::is_same<T, float>::value) {
        v[0] = __uint_as_float(w.x);
        v[1] = __uint_as_float(w.y);
        v[2] = __uint_as_float(w.z);
        v[3] = __uint_as_float(w.w);
    } else {
        const uint32_t q[4] = {w.x, w.y, w.z, w.w};
#pragma unroll
        for (int i = 0; i < 4; ++i) {
            v[2 * i] = bf_lo(q[i]);
            v[2 * i + 1] = bf_hi(q[i]);
        }
    }
#pragma unroll
    for (int i = 0; i < VEC; ++i) {
        if (!isfinite(v[i]))
            ++k;
        else
            m = fmax(m, fabs(v[i]));
    }
}

template <class T>
__global__ void k_check_partial(const T* __restrict__ u, int nplanes, GridDesc g,
                                double* __restrict__ pmax, unsigned long long* __restrict__ pcnt) {
    constexpr int VEC = 16 / sizeof(T);
    __shared__ double shm[256];
    __shared__ unsigned long long shc[256];
    double m = 0.0;
    unsigned long long k = 0;
    const long long t0 = (long long)blockIdx.x * blockDim.x + threadIdx.x;
    const long long stride = (long long)gridDim.x * blockDim.x;
    const long long nv = g.ncell / VEC, tail = g.ncell - nv * VEC;
    for (int pl = 0; pl < nplanes; ++pl) {
        const T* p = u + (long long)pl * g.pstride;
#pragma unroll 2
        for (long long j = t0; j < nv; j += stride) check_vals<T>(*(const uint4*)(p + j * VEC), m, k);
        if (t0 < tail) {
            const double v = (double)ld(p + nv * VEC + t0);
            if (!isfinite(v))
                ++k;
            else
                m = fmax(m, fabs(v));
        }
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
// The transposed substeps run on the window sweep (modes kAdjTgt/kAdjDual
// above); what remains is the chain rule from the decay factors to the
// cell-centred medium.


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

// Anisotropic scattering: the sweeps already accumulated dL/d(mean sigma_a)
// and dL/d(mean sigma_s) per grid (rows 2s, 2s + 1); only the transpose of
// the means remains.
__global__ void k_grad_final_aniso(const double* __restrict__ grad, double* __restrict__ dsa,
                                   double* __restrict__ dss, GridDesc g) {
    const long long c = (long long)blockIdx.x * blockDim.x + threadIdx.x;
    if (c >= g.ncell) return;
    double ta = 0.0, ts = 0.0;
    for (int s = 0; s < 8; ++s) {
        const int bits = c_grid_bits[s];
        const int ox = bits & 1, oy = (bits >> 1) & 1, oz = (bits >> 2) & 1;
        double aa = 0.0, as = 0.0;
        int cnt = 0;
        for (int bz = 0; bz <= oz; ++bz)
            for (int by = 0; by <= oy; ++by)
                for (int bx = 0; bx <= ox; ++bx) {
                    const long long k = shifted(c, bx, by, bz, true, g);
                    aa += grad[(long long)(2 * s) * g.ncell + k];
                    as += grad[(long long)(2 * s + 1) * g.ncell + k];
                    ++cnt;
                }
        ta += aa / cnt;
        ts += as / cnt;
    }
    if (dsa) dsa[c] = ta;
    if (dss) dss[c] = ts;
}

hipError_t launch_grad_final(const double* grad, const double* tab, const double* sa,
                             const double* ss, double* dsa, double* dss, GridDesc g, double dt,
                             bool aniso, hipStream_t st) {
    const unsigned nb = (unsigned)((g.ncell + 255) / 256);
    if (aniso)
        hipLaunchKernelGGL(k_grad_final_aniso, dim3(nb), dim3(256), 0, st, grad, dsa, dss, g);
    else
        hipLaunchKernelGGL(k_grad_final, dim3(nb), dim3(256), 0, st, grad, tab, sa, ss, dsa, dss,
                           g, dt);
    return hipGetLastError();
}

}  // namespace pm

namespace pm {

// ------------------------------------------------------------- halo faces --
// Gather (pack) or scatter (unpack) of the one-cell halo faces a sweep of
// one parity needs from its neighbours when the box is split across GPUs.
// Workgroup (x, y) takes chunk y of kHaloChunk packed elements of the
// (face, moment) pair x; a lane moves kHaloPer elements of the chunk, all
// loads issued before the stores.  Inside a face the elements follow memory
// order (fast coordinate: y for an x face, x for y and z faces), so lanes
// touch consecutive packed elements and, for y and z faces, consecutive
// cells.  Packed element end[f-1] + j area[f] + a, as the face map lists it.
constexpr int kHaloPer = 8;
constexpr int kHaloChunk = 256 * kHaloPer;

template <class T, bool UNPACK>
__global__ void __launch_bounds__(256)
k_halo(T* __restrict__ u, T* __restrict__ buf, const int* __restrict__ slots, HaloFaces hf,
       GridDesc g) {
    const int fm = blockIdx.x;  // (face, moment) pair
    int f = 0;
#pragma unroll
    for (int i = 0; i < 5; ++i) f += fm >= hf.slot0[i + 1] ? 1 : 0;
    const int area = (int)hf.area[f];
    const int a0 = blockIdx.y * kHaloChunk + threadIdx.x;
    if (a0 >= area) return;
    const int j = fm - hf.slot0[f];
    const int d = f >> 1, layer = hf.layer[f];
    const int nfast = d == 0 ? g.ny : g.nx;
    const long long start = (f == 0 ? 0 : hf.end[f - 1]) + (long long)j * area;
    T* plane = u + (long long)slots[fm] * g.pstride;
    long long cell[kHaloPer];
    T v[kHaloPer];
#pragma unroll
    for (int i = 0; i < kHaloPer; ++i) {
        const int a = a0 + i * 256;
        const int slow = a / nfast, fast = a - slow * nfast;
        if (d == 0)
            cell[i] = layer + (long long)g.nx * (fast + (long long)g.ny * slow);
        else if (d == 1)
            cell[i] = fast + (long long)g.nx * (layer + (long long)g.ny * slow);
        else
            cell[i] = fast + (long long)g.nx * (slow + (long long)g.ny * layer);
        if (a < area) v[i] = UNPACK ? buf[start + a] : plane[cell[i]];
    }
#pragma unroll
    for (int i = 0; i < kHaloPer; ++i) {
        const int a = a0 + i * 256;
        if (a >= area) break;
        if (UNPACK)
            plane[cell[i]] = v[i];
        else
            buf[start + a] = v[i];
    }
}

hipError_t launch_halo(int prec, bool unpack, void* u, void* buf, const int* slots, HaloFaces hf,
                       GridDesc g, hipStream_t st) {
    const int nfm = hf.slot0[6];
    if (nfm <= 0 || hf.end[5] <= 0) return hipSuccess;
    long long amax = 0;
    for (int f = 0; f < 6; ++f) amax = hf.area[f] > amax ? hf.area[f] : amax;
    if (amax >= (1LL << 31) - kHaloChunk || nfm > (1 << 30)) return hipErrorInvalidValue;
    const long long ny = (amax + kHaloChunk - 1) / kHaloChunk;
    if (ny > 65535) return hipErrorInvalidValue;  // grid y limit
    const dim3 grid((unsigned)nfm, (unsigned)ny), block(256);
#define PM_HALO(T)                                                                               \
    if (unpack)                                                                                  \
        hipLaunchKernelGGL((k_halo<T, true>), grid, block, 0, st, (T*)u, (T*)buf, slots, hf, g); \
    else                                                                                         \
        hipLaunchKernelGGL((k_halo<T, false>), grid, block, 0, st, (T*)u, (T*)buf, slots, hf, g);
    if (prec == kF64) {
        PM_HALO(double)
    } else if (prec == kF32) {
        PM_HALO(float)
    } else {
        PM_HALO(bf16s)
    }
#undef PM_HALO
    return hipGetLastError();
}

}  // namespace pm
