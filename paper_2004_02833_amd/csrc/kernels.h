// Device-side data structures and launchers of libpm (internal).
#pragma once
#include <hip/hip_runtime.h>

#include <cstdint>

namespace pm {

enum Prec { kF64 = 0, kF32 = 1, kBF16 = 2 };

// Table rows (float64 planes of ncell values): alpha/beta of grid g in rows
// 2g and 2g+1 (g in storage order; tau = dt/2 on odd grids, dt on even
// grids), moment 0 in rows 16/17, q in row 18, and alpha/beta of the odd
// grids for a full step tau = dt in rows 19 + 2f, 20 + 2f (f = g - 4), used
// when two odd half steps of consecutive steps are merged.
constexpr int kTabRows = 27;
constexpr int kTabMom0 = 16;
constexpr int kTabQ = 18;
constexpr int kTabOddFull = 19;
// Gradient accumulators: rows 2s (d/d alpha) and 2s+1 (d/d beta), s = 0..8
// (grid g -> s = g, moment 0 -> s = 8).
constexpr int kGradRows = 18;

struct GridDesc {
    int nx, ny, nz;
    long long ncell;
    long long pstride;  // elements between consecutive moment planes
};

// Window sweep (see kernels.hip).  A sweep of one parity is split into
// passes of K target degrees; pass p, source column mu (0 <= mu <= N + 2)
// is described by host-built streams, in the order the kernel consumes them:
//   src[((p * MU1 + mu) * (K + 1) + b) * 2 + ty] = {slot or -1, parity bits}
//       (slots count from the first plane of the dual parity; targets from
//       the first plane of the sweep's parity)
//       source degree L0 - 1 + 2b, m = +mu (ty 0, cos) or -mu (ty 1, sin);
//   tgt[((p * MU1 + mu) * K + t) * 2 + ty] = {slot or -1, alpha table row}
//       target degree L0 + 2t, m = +-mu;
//   coef[(((p * MU1 + mu) * (K + 1) + b) * 2 + ty) * 2 + side) * 5 + r]
//       coupling of that source (column mu) to the targets of degree
//       ls + 1 (side 0) or ls - 1 (side 1):
//       r = 0: x to column mu-1 (same type)   1: y to column mu-1 (other type)
//           2: z to column mu (same m)        3: x to column mu+1   4: y to column mu+1
//       value K = s * M_d[i, j] / dx (s = +1 if the source is unstaggered in
//       d, else -1), zero where the target does not exist.
// with MU1 = N + 3 (source columns 0..N+1 and an empty column N+2, so the
// next column can always be requested) and L0 = parity + 2 K p.
struct WinArgs {
    int N;
    int parity;   // parity (l mod 2) of the target moments
    int K;        // target degrees per pass
    int npass;
    const int2* src;
    const int2* tgt;
    const void* coef;  // values of the accumulation type
};

// Target degrees per pass of the forward sweeps (for a storage precision,
// row length nx, moment order N and anisotropic scattering) and of the
// transposed ones (pm_grad).
int win_depth(int prec, int nx, int N, bool aniso);
int adj_depth(int prec);

// Anisotropic scattering: gl = device array of g_0 .. g_N (g_0 = 1), or
// nullptr for the isotropic tables; tau = length of the substep.
struct Aniso {
    const double* gl;
    double tau;
};

// aniso: rows 2s, 2s + 1 hold the means of sigma_a and sigma_s on grid s
// (s in storage order) and row kTabQ holds q; the other rows are unused.
hipError_t launch_tables(const double* sa, const double* ss, const double* q, double* tab,
                         GridDesc g, double dt, bool aniso, hipStream_t st);
// float copy of the isotropic tables: gamma = 1 - alpha in every alpha row,
// the other rows rounded (kTabRows rows of n values)
hipError_t launch_tables_f32(const double* tab, float* tabf, long long n, hipStream_t st);

// Planes of a sweep, as element offsets from one base pointer (the pool):
// src = first plane of the dual parity (the sources), tin / tout = first
// target plane read / written (equal for an update in place); for the
// target side of the transpose also aux = first target plane of the old
// state and w = first plane of the output beta * lam.  Slot numbers in the
// streams count from the first plane of their parity.
struct StateOffs {
    long long src, tin, tout, aux, w;
};

// rowbase: table row of alpha for the first target grid of the parity
// (0 for the even sweep, 8 for an odd half step, kTabOddFull for a full one;
// with anisotropic scattering 0 or 8, the substep length coming from an.tau).
// tabf: float copy of the tables (launch_tables_f32) read by the FP32
// update of float and bfloat16 storage with isotropic scattering (nullptr
// otherwise).
hipError_t launch_sweep_win(int prec, void* pool, StateOffs so, const double* tab, const float* tabf,
                            int rowbase, Aniso an, WinArgs a, GridDesc g, hipStream_t st);

// Transposed substep on the window streams.  side 0 (target side): so.src /
// so.aux = dual / target half of the old state, tin = tout = cotangent lam
// of the targets (updated), w = output beta * lam, gp = per-pass gradient
// rows of this parity ([npass][kGradRows][ncell], added to).  side 1 (dual
// side): src = the w half, tin = tout = lam of the dual moments.  FP64 and
// FP32 only.  With anisotropic scattering the gradient rows 2s and 2s + 1
// are dL/d(mean sigma_a) and dL/d(mean sigma_s) of grid s.
hipError_t launch_adj_win(int prec, int side, void* pool, StateOffs so, double* gp,
                          const double* tab, int rowbase, Aniso an, WinArgs a, GridDesc g,
                          hipStream_t st);
hipError_t launch_grad_sum(const double* gp, int nbuf, double* grad, long long n, hipStream_t st);

hipError_t launch_to_f64(int prec, const void* src_plane, double* dst, long long n,
                         hipStream_t st);
hipError_t launch_from_f64(int prec, const double* src, void* dst_plane, long long n,
                           hipStream_t st);

// sum of moment-0 plane into *out (device double), two-pass deterministic.
hipError_t launch_sum(int prec, const void* plane, long long n, double* partial, int npart,
                      double* out, hipStream_t st);
// max |u| and non-finite count over nplanes planes.
hipError_t launch_check(int prec, const void* u, int nplanes, GridDesc g, double* pmax,
                        unsigned long long* pcount, int npart, double* out_max,
                        unsigned long long* out_count, hipStream_t st);

hipError_t launch_grad_final(const double* grad, const double* tab, const double* sa,
                             const double* ss, double* dsa, double* dss, GridDesc g, double dt,
                             bool aniso, hipStream_t st);

hipError_t launch_fill_zero(void* p, long long bytes, hipStream_t st);

// Device address of the library's static scratch array on the current
// device (taken once per device with hipGetSymbolAddress), and the number of
// reduction partials it holds (that many doubles, then that many unsigned
// long longs).
hipError_t scratch_device(void** ptr);
int scratch_partials();

// Halo faces of a sweep, in packing order x-, x+, y-, y+, z-, z+: face f
// holds the layer `layer[f]` of the moments whose slots are
// slots[slot0[f] .. slot0[f + 1]) (area[f] cells each; slot0[6] = all
// moments); end[f] = packed elements of faces 0..f.
struct HaloFaces {
    long long end[6];
    long long area[6];
    int layer[6];
    int slot0[7];
};
hipError_t launch_halo(int prec, bool unpack, void* u, void* buf, const int* slots, HaloFaces hf,
                       GridDesc g, hipStream_t st);

}  // namespace pm
