// C ABI of libpm: context management, validation and the step driver.
//
// A time step is the Strang composition of eq. (6): the odd-grid half step,
// the even-grid full step and the odd-grid half step, each one sweep launch
// on the bound stream (paper Sec. 2.1 and Sec. 3.2, where a step is the
// sweeps S^o, S^e, S^o).  The gradient pass walks the recorded steps
// backwards from device checkpoints (the paper has no derivatives; this is
// the transpose of the discrete step).
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdio>
#include <cstring>
#include <string>
#include <unordered_map>
#include <utility>
#include <vector>

#include "../../include/pm.h"
#include "kernels.h"
#include "pm_internal.h"

namespace {

std::string g_err = "no error";
int g_pending_prec = PM_FP64;
std::vector<double> g_pending_scat;  // g_1, g_2, ... for the next pm_init
int g_merge = 1;
hipStream_t g_bound = nullptr;  // caller's stream (nullptr: own stream)

int fail(int code, const std::string& msg) {
    g_err = msg;
    return code;
}

#define HIPCHK(x)                                                                   \
    do {                                                                            \
        hipError_t e_ = (x);                                                        \
        if (e_ != hipSuccess)                                                       \
            return fail(e_ == hipErrorOutOfMemory ? PM_ENOMEM : PM_EDEVICE,         \
                        std::string(#x) + ": " + hipGetErrorString(e_));            \
    } while (0)

size_t elem_size(int prec) { return prec == PM_FP64 ? 8 : prec == PM_FP32 ? 4 : 2; }

// Halo faces of the sweeps of one parity (see halo_plan).
struct HaloPlan {
    std::vector<int> slots;  // slots of the faces' moments, face after face
    pm::HaloFaces hf{};
};

struct Ctx {
    bool live = false;
    int N = 0, V = 0, nx = 0, ny = 0, nz = 0;
    long long ncell = 0;
    double h[3] = {0, 0, 0};  // cell edges dx, dy, dz
    double dt = 0;
    int prec = PM_FP64;
    size_t esz = 8;
    pm::GridDesc g{};
    pm::Layout L;
    long long ve = 0;  // planes of the even parity (slots [0, ve)); odd ones follow
    void* u = nullptr;
    double* tab = nullptr;
    float* tabf = nullptr;  // float copy for the FP32 update (float/bfloat16 storage, isotropic)
    double* sig = nullptr;  // sigma_a, sigma_s (device copies)
    bool aniso = false;     // some g_l != 0 for 1 <= l <= N
    double* gl = nullptr;   // g_0 .. g_N on the device (anisotropic scattering)
    void* win_mem = nullptr;  // window sweep streams (both parities)
    HaloPlan halo[2];         // halo faces of the sweeps of each parity
    int* halo_slots[2] = {nullptr, nullptr};
    void* adj_mem = nullptr;  // streams of the transposed sweeps when their depth differs
    pm::WinArgs win[2]{};     // forward sweeps
    pm::WinArgs wadj[2]{};    // transposed sweeps (pm_grad)
    double* plane64 = nullptr;
    double* red = nullptr;
    unsigned long long* redc = nullptr;
    int npart = 256;   // partial sums of pm_total (its rounding depends on it)
    int ncheck = 1024; // partial results of pm_check / pm_check_noalloc
    hipStream_t own = nullptr;
    int cfl_warn = 0;
    int ck = 0;
    long long rec_steps = 0;
    std::vector<void*> ckpts;
    bool timing = false;
    std::vector<std::pair<hipEvent_t, hipEvent_t>> ev[2];
    long long dev_bytes = 0;
    long long base_bytes = 0;

    size_t state_bytes() const { return (size_t)V * (size_t)g.pstride * esz; }
    // element offset of the first plane of a parity within a state
    long long half(int parity) const { return parity ? ve * g.pstride : 0; }
    hipStream_t stream() const { return g_bound ? g_bound : own; }
    void* plane(void* base, int slot) const {
        return (char*)base + (size_t)slot * (size_t)g.pstride * esz;
    }
};

Ctx C;

template <class P>
int dmalloc(P** p, size_t bytes, const char* what) {
    void* q = nullptr;
    hipError_t e = hipMalloc(&q, bytes ? bytes : 1);
    if (e != hipSuccess) {
        (void)hipGetLastError();
        return fail(e == hipErrorOutOfMemory ? PM_ENOMEM : PM_EDEVICE,
                    std::string("hipMalloc(") + what + ", " + std::to_string(bytes) +
                        " bytes): " + hipGetErrorString(e));
    }
    C.dev_bytes += (long long)bytes;
    *p = (P*)q;
    return PM_OK;
}

void dfree(void* p) {
    if (p) (void)hipFree(p);
}

// Identifies the recorded forward: changes whenever the recording starts,
// stops, is dropped or is extended by pm_step (pm_recording_id).
long long g_rec_id = 1;

void drop_recording() {
    for (void* p : C.ckpts) dfree(p);
    C.ckpts.clear();
    C.rec_steps = 0;
    ++g_rec_id;
}

void drop_events() {
    for (auto& v : C.ev)
        for (auto& pr : v) {
            (void)hipEventDestroy(pr.first);
            (void)hipEventDestroy(pr.second);
        }
    C.ev[0].clear();
    C.ev[1].clear();
}

void release() {
    drop_recording();
    drop_events();
    dfree(C.u);
    dfree(C.tab);
    dfree(C.tabf);
    dfree(C.sig);
    dfree(C.gl);
    dfree(C.win_mem);
    dfree(C.halo_slots[0]);
    dfree(C.halo_slots[1]);
    dfree(C.adj_mem);
    dfree(C.plane64);
    dfree(C.red);
    dfree(C.redc);
    if (C.own) (void)hipStreamDestroy(C.own);
    C = Ctx();
}

bool finite_nonneg(const double* a, long long n, const char* name, std::string& msg) {
    for (long long i = 0; i < n; ++i)
        if (!std::isfinite(a[i]) || a[i] < 0.0) {
            msg = std::string(name) + "[" + std::to_string(i) + "] is negative or not finite";
            return false;
        }
    return true;
}

// Plane stride: a multiple of 64 elements, padded so that consecutive planes
// do not sit at power-of-two distances.
long long plane_stride(long long ncell) {
    long long s = (ncell + 63) / 64 * 64;
    if ((s & (s - 1)) == 0 && s >= 4096) s += 64;
    return s;
}

// Streams of the window sweep (layout documented in kernels.h).  Every
// nonzero flux entry with a target of the sweep's parity must land in exactly
// one coefficient slot; the count is checked.
int build_window_tables(int K, pm::WinArgs (&win)[2], void** mem) {
    const pm::Layout& L = C.L;
    // columns mu = 0..N+1 and one empty column N+2: a sweep requests the next
    // column's sources unconditionally
    const int N = C.N, V = C.V, MU1 = N + 3;
    std::unordered_map<long long, double> flux;
    long long nnz_par[2] = {0, 0};
    for (const pm::FluxEntry& e : pm::flux_entries(N)) {
        flux[((long long)e.row * V + e.col) * 3 + e.dir] = e.val;
        int l, m;
        pm::moment_lm(e.row, l, m);
        ++nnz_par[l & 1];
    }
    auto exists = [&](int l, int mu, int ty) {
        return l >= 0 && l <= N && mu >= 0 && mu <= l && !(ty == 1 && mu == 0);
    };
    auto idx = [](int l, int mu, int ty) { return l * l + l + (ty == 0 ? mu : -mu); };
    struct Host {
        std::vector<int2> src, tgt;
        std::vector<double> coef;
    } H[2];
    for (int p = 0; p < 2; ++p) {
        const int npass = N >= p ? (N - p) / (2 * K) + 1 : 0;
        win[p].N = N;
        win[p].parity = p;
        win[p].K = K;
        win[p].npass = npass;
        Host& h = H[p];
        h.src.assign((size_t)npass * MU1 * (K + 1) * 2, make_int2(-1, 0));
        h.tgt.assign((size_t)npass * MU1 * K * 2, make_int2(-1, 0));
        h.coef.assign((size_t)npass * MU1 * (K + 1) * 20, 0.0);
        long long used = 0;
        for (int pass = 0; pass < npass; ++pass) {
            const int L0 = p + 2 * K * pass;
            for (int mu = 0; mu < MU1; ++mu) {
                for (int b = 0; b <= K; ++b)
                    for (int ty = 0; ty < 2; ++ty) {
                        const int ls = L0 - 1 + 2 * b;
                        if (!exists(ls, mu, ty)) continue;
                        const int j = idx(ls, mu, ty);
                        const int bits = pm::grid_bits(ls, ty == 0 ? mu : -mu);
                        h.src[((size_t)(pass * MU1 + mu) * (K + 1) + b) * 2 + ty] =
                            make_int2(L.slot_of[j] - (p ? 0 : (int)C.ve), bits);
                        for (int side = 0; side < 2; ++side) {
                            const int t = side == 0 ? b : b - 1;
                            if (t < 0 || t >= K) continue;
                            const int lt = L0 + 2 * t;
                            // (target column, target type, direction) of the five roles
                            const int tmu[5] = {mu - 1, mu - 1, mu, mu + 1, mu + 1};
                            const int tty[5] = {ty, 1 - ty, ty, ty, 1 - ty};
                            const int dir[5] = {0, 1, 2, 0, 1};
                            for (int r = 0; r < 5; ++r) {
                                if (!exists(lt, tmu[r], tty[r])) continue;
                                const int i = idx(lt, tmu[r], tty[r]);
                                auto it = flux.find(((long long)i * V + j) * 3 + dir[r]);
                                if (it == flux.end()) continue;
                                const double sgn = ((bits >> dir[r]) & 1) ? -1.0 : 1.0;
                                h.coef[((((size_t)(pass * MU1 + mu) * (K + 1) + b) * 2 + ty) * 2 + side) * 5 + r] =
                                    sgn * it->second / C.h[dir[r]];
                                ++used;
                            }
                        }
                    }
                for (int t = 0; t < K; ++t)
                    for (int ty = 0; ty < 2; ++ty) {
                        const int lt = L0 + 2 * t;
                        if (!exists(lt, mu, ty)) continue;
                        const int i = idx(lt, mu, ty);
                        const int row = i == 0 ? pm::kTabMom0 : 2 * L.order_of[i];
                        h.tgt[((size_t)(pass * MU1 + mu) * K + t) * 2 + ty] =
                            make_int2(L.slot_of[i] - (p ? (int)C.ve : 0), row);
                    }
            }
        }
        if (used != nnz_par[p])
            return fail(PM_EINVAL, "internal: window streams cover " + std::to_string(used) + " of " +
                                       std::to_string(nnz_par[p]) + " couplings");
        // slots count from the first plane of their parity half
        const long long nhalf[2] = {C.ve, (long long)V - C.ve};
        for (const int2& e : h.src)
            if (e.x >= nhalf[1 - p]) return fail(PM_EINVAL, "internal: source slot outside its half");
        for (const int2& e : h.tgt)
            if (e.x >= nhalf[p]) return fail(PM_EINVAL, "internal: target slot outside its half");
    }
    const bool f64 = C.prec == PM_FP64;
    const size_t es = f64 ? sizeof(double) : sizeof(float);
    auto up = [](size_t x) { return (x + 255) / 256 * 256; };
    size_t total = 0, off[2][3];
    for (int p = 0; p < 2; ++p) {
        off[p][0] = total; total += up(H[p].src.size() * sizeof(int2));
        off[p][1] = total; total += up(H[p].tgt.size() * sizeof(int2));
        off[p][2] = total; total += up(H[p].coef.size() * es);
    }
    int rc = dmalloc(mem, total, "window streams");
    if (rc) return rc;
    char* base = (char*)*mem;
    for (int p = 0; p < 2; ++p) {
        if (!H[p].src.empty())
            HIPCHK(hipMemcpy(base + off[p][0], H[p].src.data(), H[p].src.size() * sizeof(int2), hipMemcpyHostToDevice));
        if (!H[p].tgt.empty())
            HIPCHK(hipMemcpy(base + off[p][1], H[p].tgt.data(), H[p].tgt.size() * sizeof(int2), hipMemcpyHostToDevice));
        if (!H[p].coef.empty()) {
            if (f64) {
                HIPCHK(hipMemcpy(base + off[p][2], H[p].coef.data(), H[p].coef.size() * es, hipMemcpyHostToDevice));
            } else {
                std::vector<float> c32(H[p].coef.begin(), H[p].coef.end());
                HIPCHK(hipMemcpy(base + off[p][2], c32.data(), c32.size() * es, hipMemcpyHostToDevice));
            }
        }
        win[p].src = (const int2*)(base + off[p][0]);
        win[p].tgt = (const int2*)(base + off[p][1]);
        win[p].coef = base + off[p][2];
    }
    return PM_OK;
}

// One sweep of the given parity; `full` selects tau = dt for the odd grids
// (two merged odd half steps).
int sweep(void* u, int parity, bool full = false) {
    if (C.win[parity].npass == 0) return PM_OK;
    hipEvent_t a = nullptr, b = nullptr;
    if (C.timing) {
        HIPCHK(hipEventCreate(&a));
        HIPCHK(hipEventCreate(&b));
        HIPCHK(hipEventRecord(a, C.stream()));
    }
    const double tau = parity == 0 || full ? C.dt : 0.5 * C.dt;
    const int rowbase = parity == 0 ? 0 : full && !C.aniso ? pm::kTabOddFull : 8;
    const pm::Aniso an{C.aniso ? C.gl : nullptr, tau};
    const pm::StateOffs so{C.half(1 - parity), C.half(parity), C.half(parity), 0, 0};
    HIPCHK(pm::launch_sweep_win(C.prec, u, so, C.tab, C.tabf, rowbase, an, C.win[parity], C.g, C.stream()));
    if (C.timing) {
        HIPCHK(hipEventRecord(b, C.stream()));
        C.ev[parity].push_back({a, b});
    }
    return PM_OK;
}

int full_step(void* u) {
    int rc;
    if ((rc = sweep(u, 1))) return rc;
    if ((rc = sweep(u, 0))) return rc;
    return sweep(u, 1);
}

// n steps of eq. (6).  With merging, the trailing odd half step of a step
// and the leading one of the next see the same (unchanged) even moments and
// the odd moments carry no source, so together they are one odd substep of
// length dt (alpha_h^2 = alpha_dt, beta_h (1 + alpha_h) = beta_dt): n steps
// take 2n + 1 sweeps instead of 3n.  The result differs by rounding only.
int run_steps(void* u, long long n, bool merged) {
    if (n <= 0) return PM_OK;
    if (!merged) {
        for (long long s = 0; s < n; ++s) {
            int rc = full_step(u);
            if (rc) return rc;
        }
        return PM_OK;
    }
    int rc;
    if ((rc = sweep(u, 1))) return rc;
    for (long long s = 0; s < n; ++s) {
        if ((rc = sweep(u, 0))) return rc;
        if ((rc = sweep(u, 1, s + 1 < n))) return rc;
    }
    return PM_OK;
}

// Halo faces of a sweep of parity p when the box is one GPU's share of a
// split grid.  The sweep reads each dual moment (parity 1 - p) at one
// neighbour per direction d: forward (c + e_d) when the moment is
// unstaggered in d, backward when it is staggered.  So the -d neighbour
// needs this box's layer 0 of the dual moments unstaggered in d (face d-)
// and the +d neighbour its last layer of those staggered in d (face d+).
// Packing order: faces x-, x+, y-, y+, z-, z+; in a face the moments by
// storage slot, then the face cells with the two other coordinates in
// memory order.
HaloPlan halo_plan(const pm::Layout& L, int nx, int ny, int nz, int parity) {
    HaloPlan hp;
    const long long n[3] = {nx, ny, nz};
    long long end = 0;
    for (int f = 0; f < 6; ++f) {
        const int d = f >> 1, side = f & 1;
        hp.hf.slot0[f] = (int)hp.slots.size();
        for (int s = 0; s < L.V; ++s) {
            const int i = L.moment_of[s];
            int l, m;
            pm::moment_lm(i, l, m);
            if ((l & 1) != 1 - parity) continue;
            if (((pm::grid_bits(l, m) >> d) & 1) != side) continue;
            hp.slots.push_back(s);
        }
        const long long cnt = (long long)hp.slots.size() - hp.hf.slot0[f];
        hp.hf.area[f] = n[(d + 1) % 3] * n[(d + 2) % 3];
        hp.hf.layer[f] = side ? (int)n[d] - 1 : 0;
        end += cnt * hp.hf.area[f];
        hp.hf.end[f] = end;
    }
    hp.hf.slot0[6] = (int)hp.slots.size();
    return hp;
}

// The faces of the directions in `dirs` (bit d: direction d split across
// GPUs): the others get no cells, and the packed offsets close up.
pm::HaloFaces halo_masked(pm::HaloFaces hf, int dirs) {
    long long end = 0;
    for (int f = 0; f < 6; ++f) {
        const long long cnt = hf.slot0[f + 1] - hf.slot0[f];
        if (!((dirs >> (f >> 1)) & 1)) hf.area[f] = 0;
        end += cnt * hf.area[f];
        hf.end[f] = end;
    }
    return hf;
}

int check_moment(int moment) {
    if (!C.live) return fail(PM_ESTATE, "no context: call pm_init first");
    if (moment < 0 || moment >= C.V)
        return fail(PM_EINVAL, "moment " + std::to_string(moment) + " out of range [0, " +
                                   std::to_string(C.V) + ")");
    return PM_OK;
}

}  // namespace

extern "C" {

int pm_set_precision(int p) {
    if (p != PM_FP64 && p != PM_FP32 && p != PM_BF16)
        return fail(PM_EINVAL, "unknown precision " + std::to_string(p));
    g_pending_prec = p;
    return PM_OK;
}

int pm_set_scattering(const double* g, int count) {
    if (count < 0 || count > PM_N_MAX)
        return fail(PM_EINVAL, "scattering count must be in [0, " + std::to_string(PM_N_MAX) + "]");
    if (count > 0 && !g) return fail(PM_EINVAL, "scattering moments are NULL");
    for (int l = 0; l < count; ++l)
        if (!std::isfinite(g[l]) || g[l] < -1.0 || g[l] > 1.0)
            return fail(PM_EINVAL, "g[" + std::to_string(l) + "] (degree " + std::to_string(l + 1) +
                                       ") is not finite or outside [-1, 1]");
    g_pending_scat.assign(g, g + count);
    return PM_OK;
}

int pm_init(int N, int nx, int ny, int nz, double dx, double dt, const double* sigma_a,
            const double* sigma_s, const double* q) {
    return pm_init_cells(N, nx, ny, nz, dx, dx, dx, dt, sigma_a, sigma_s, q);
}

int pm_init_cells(int N, int nx, int ny, int nz, double dx, double dy, double dz, double dt,
                  const double* sigma_a, const double* sigma_s, const double* q) {
    if (N < 0 || N > PM_N_MAX) return fail(PM_EINVAL, "N must be in [0, 63]");
    if (nx < 1 || ny < 1 || nz < 1) return fail(PM_EINVAL, "grid sizes must be >= 1");
    const long long ncell = (long long)nx * ny * nz;
    if (ncell >= (1LL << 31)) return fail(PM_EINVAL, "more than 2^31 - 1 cells");
    for (double hd : {dx, dy, dz})
        if (!(hd > 0.0) || !std::isfinite(hd))
            return fail(PM_EINVAL, "cell edges dx, dy, dz must be positive and finite");
    if (!(dt > 0.0) || !std::isfinite(dt)) return fail(PM_EINVAL, "dt must be positive and finite");
    if (!sigma_a || !sigma_s) return fail(PM_EINVAL, "sigma_a and sigma_s are required");
    std::string msg;
    if (!finite_nonneg(sigma_a, ncell, "sigma_a", msg) || !finite_nonneg(sigma_s, ncell, "sigma_s", msg))
        return fail(PM_EINVAL, msg);
    if (q)
        for (long long i = 0; i < ncell; ++i)
            if (!std::isfinite(q[i])) return fail(PM_EINVAL, "q[" + std::to_string(i) + "] not finite");

    release();
    C.N = N;
    C.V = (N + 1) * (N + 1);
    C.nx = nx;
    C.ny = ny;
    C.nz = nz;
    C.ncell = ncell;
    C.h[0] = dx;
    C.h[1] = dy;
    C.h[2] = dz;
    C.dt = dt;
    C.prec = g_pending_prec;
    C.esz = elem_size(C.prec);
    C.g.nx = nx;
    C.g.ny = ny;
    C.g.nz = nz;
    C.g.ncell = ncell;
    C.g.pstride = plane_stride(ncell);
    C.L = pm::make_layout(N);
    C.ve = 0;
    for (int l = 0; l <= N; l += 2) C.ve += 2 * l + 1;
    std::vector<double> gl(N + 1, 0.0);
    gl[0] = 1.0;
    for (int l = 1; l <= N && l - 1 < (int)g_pending_scat.size(); ++l) gl[l] = g_pending_scat[l - 1];
    C.aniso = std::any_of(gl.begin() + 1, gl.end(), [](double v) { return v != 0.0; });
    // sigma = 0 Fourier symbol: stable iff dt * lambda_max * sqrt(sum_d 1/h_d^2) <= 1
    const double lim =
        N > 0 ? 1.0 / (pm::lambda_max(N) * std::sqrt(1.0 / (dx * dx) + 1.0 / (dy * dy) + 1.0 / (dz * dz)))
              : INFINITY;
    C.cfl_warn = dt > lim ? 1 : 0;

    int rc;
    hipError_t e = hipStreamCreate(&C.own);
    if (e != hipSuccess) {
        C.own = nullptr;
        release();
        return fail(PM_EDEVICE, std::string("hipStreamCreate: ") + hipGetErrorString(e));
    }
#define TRY(x)            \
    do {                  \
        rc = (x);         \
        if (rc) {         \
            release();    \
            return rc;    \
        }                 \
    } while (0)
    {
        size_t fr = 0, tot = 0;
        hipError_t me = hipMemGetInfo(&fr, &tot);
        const size_t need = C.state_bytes() + sizeof(double) * (pm::kTabRows + 3) * (size_t)ncell +
                            (C.prec != PM_FP64 && !C.aniso ? sizeof(float) * pm::kTabRows * (size_t)ncell : 0);
        if (me != hipSuccess) {
            release();
            return fail(PM_EDEVICE, std::string("hipMemGetInfo: ") + hipGetErrorString(me));
        }
        if (need > fr) {
            release();
            return fail(PM_ENOMEM, "context needs " + std::to_string(need) + " bytes, " +
                                       std::to_string(fr) + " free on the device");
        }
    }
    TRY(dmalloc(&C.u, C.state_bytes(), "state"));
    TRY(dmalloc(&C.tab, sizeof(double) * pm::kTabRows * (size_t)ncell, "tables"));
    TRY(dmalloc(&C.sig, sizeof(double) * 2 * (size_t)ncell, "sigma"));
    const bool ftab = C.prec != PM_FP64 && !C.aniso;
    if (ftab) TRY(dmalloc(&C.tabf, sizeof(float) * pm::kTabRows * (size_t)ncell, "float tables"));
    if (C.aniso) TRY(dmalloc(&C.gl, sizeof(double) * gl.size(), "scattering moments"));
    TRY(dmalloc(&C.plane64, sizeof(double) * (size_t)ncell, "plane"));
    TRY(dmalloc(&C.red, sizeof(double) * (std::max(C.npart, C.ncheck) + 1), "reduction"));
    TRY(dmalloc(&C.redc, sizeof(unsigned long long) * (C.ncheck + 1), "reduction"));
    const int kwin = pm::win_depth(C.prec, nx, N, C.aniso);
    TRY(build_window_tables(kwin, C.win, &C.win_mem));

    if (C.prec != PM_BF16 && pm::adj_depth(C.prec) != kwin) {
        TRY(build_window_tables(pm::adj_depth(C.prec), C.wadj, &C.adj_mem));
    } else {
        C.wadj[0] = C.win[0];
        C.wadj[1] = C.win[1];
    }
    hipStream_t s = C.stream();
    auto dev = [&](hipError_t err, const char* what) -> int {
        if (err == hipSuccess) return PM_OK;
        return fail(PM_EDEVICE, std::string(what) + ": " + hipGetErrorString(err));
    };
    for (int p = 0; p < 2; ++p) {
        C.halo[p] = halo_plan(C.L, nx, ny, nz, p);
        TRY(dmalloc(&C.halo_slots[p], sizeof(int) * std::max<size_t>(1, C.halo[p].slots.size()), "halo faces"));
        if (!C.halo[p].slots.empty())
            TRY(dev(hipMemcpyAsync(C.halo_slots[p], C.halo[p].slots.data(), sizeof(int) * C.halo[p].slots.size(),
                                   hipMemcpyHostToDevice, C.stream()),
                    "copy halo faces"));
    }
    TRY(dev(hipMemcpyAsync(C.sig, sigma_a, sizeof(double) * ncell, hipMemcpyHostToDevice, s), "copy sigma_a"));
    TRY(dev(hipMemcpyAsync(C.sig + ncell, sigma_s, sizeof(double) * ncell, hipMemcpyHostToDevice, s), "copy sigma_s"));
    if (q) TRY(dev(hipMemcpyAsync(C.plane64, q, sizeof(double) * ncell, hipMemcpyHostToDevice, s), "copy q"));
    if (C.aniso)
        TRY(dev(hipMemcpyAsync(C.gl, gl.data(), sizeof(double) * gl.size(), hipMemcpyHostToDevice, s),
                "copy scattering moments"));
    TRY(dev(pm::launch_tables(C.sig, C.sig + ncell, q ? C.plane64 : nullptr, C.tab, C.g, dt, C.aniso, s),
            "tables"));
    if (ftab) TRY(dev(pm::launch_tables_f32(C.tab, C.tabf, ncell, s), "float tables"));
    TRY(dev(pm::launch_fill_zero(C.u, (long long)C.state_bytes(), s), "zero state"));
    TRY(dev(hipStreamSynchronize(s), "sync"));
#undef TRY
    C.base_bytes = C.dev_bytes;
    C.live = true;
    return PM_OK;
}

int pm_write(int moment, const double* src) {
    int rc = check_moment(moment);
    if (rc) return rc;
    if (!src) return fail(PM_EINVAL, "src is NULL");
    hipStream_t s = C.stream();
    const int slot = C.L.slot_of[moment];
    if (C.prec == PM_FP64) {
        HIPCHK(hipMemcpyAsync(C.plane(C.u, slot), src, sizeof(double) * C.ncell, hipMemcpyHostToDevice, s));
    } else {
        HIPCHK(hipMemcpyAsync(C.plane64, src, sizeof(double) * C.ncell, hipMemcpyHostToDevice, s));
        HIPCHK(pm::launch_from_f64(C.prec, C.plane64, C.plane(C.u, slot), C.ncell, s));
    }
    HIPCHK(hipStreamSynchronize(s));
    drop_recording();
    return PM_OK;
}

int pm_write_dev(int moment, const void* dsrc) {
    int rc = check_moment(moment);
    if (rc) return rc;
    if (!dsrc) return fail(PM_EINVAL, "src is NULL");
    const int slot = C.L.slot_of[moment];
    HIPCHK(pm::launch_from_f64(C.prec, (const double*)dsrc, C.plane(C.u, slot), C.ncell, C.stream()));
    drop_recording();
    return PM_OK;
}

int pm_step(int nsteps) {
    if (!C.live) return fail(PM_ESTATE, "no context: call pm_init first");
    if (nsteps < 0) return fail(PM_EINVAL, "nsteps < 0");
    int rc;
    long long done = 0;
    while (done < nsteps) {
        long long chunk = nsteps - done;
        if (C.ck > 0) {
            if (C.rec_steps % C.ck == 0) {
                size_t fr = 0, tot = 0;
                HIPCHK(hipMemGetInfo(&fr, &tot));
                if (C.state_bytes() > fr) return fail(PM_ENOMEM, "no device memory for a checkpoint");
                void* p = nullptr;
                if ((rc = dmalloc(&p, C.state_bytes(), "checkpoint"))) return rc;
                C.ckpts.push_back(p);
                HIPCHK(hipMemcpyAsync(p, C.u, C.state_bytes(), hipMemcpyDeviceToDevice, C.stream()));
            }
            chunk = std::min<long long>(chunk, C.ck - C.rec_steps % C.ck);  // stop at the next checkpoint
        }
        if ((rc = run_steps(C.u, chunk, g_merge != 0))) return rc;
        done += chunk;
        if (C.ck > 0) C.rec_steps += chunk;
    }
    if (C.ck > 0 && nsteps > 0) ++g_rec_id;
    return PM_OK;
}

int pm_set_merge(int on) {
    if (on != 0 && on != 1) return fail(PM_EINVAL, "pm_set_merge takes 0 or 1");
    g_merge = on;
    return PM_OK;
}

int pm_read(int moment, double* dst) {
    int rc = check_moment(moment);
    if (rc) return rc;
    if (!dst) return fail(PM_EINVAL, "dst is NULL");
    hipStream_t s = C.stream();
    const int slot = C.L.slot_of[moment];
    if (C.prec == PM_FP64) {
        HIPCHK(hipMemcpyAsync(dst, C.plane(C.u, slot), sizeof(double) * C.ncell, hipMemcpyDeviceToHost, s));
    } else {
        HIPCHK(pm::launch_to_f64(C.prec, C.plane(C.u, slot), C.plane64, C.ncell, s));
        HIPCHK(hipMemcpyAsync(dst, C.plane64, sizeof(double) * C.ncell, hipMemcpyDeviceToHost, s));
    }
    HIPCHK(hipStreamSynchronize(s));
    return PM_OK;
}

int pm_read_dev(int moment, void* ddst) {
    int rc = check_moment(moment);
    if (rc) return rc;
    if (!ddst) return fail(PM_EINVAL, "dst is NULL");
    const int slot = C.L.slot_of[moment];
    HIPCHK(pm::launch_to_f64(C.prec, C.plane(C.u, slot), (double*)ddst, C.ncell, C.stream()));
    return PM_OK;
}

int pm_set_checkpoint(int k) {
    if (k < 0) return fail(PM_EINVAL, "checkpoint interval < 0");
    if (!C.live) return fail(PM_ESTATE, "no context: call pm_init first");
    if (k > 0 && C.prec == PM_BF16)
        return fail(PM_EINVAL, "gradients are not supported for bfloat16 storage");
    drop_recording();
    C.ck = k;
    return PM_OK;
}

// Reverse pass.  One pool holds lam, w and the states of a segment as
// parity halves: a substep writes the new half of its own parity into a fresh
// buffer and shares the other half with its input, so the recomputation of a
// segment keeps every intermediate substep state without copies.  For step
// j of a segment with state (E_j, O_j): O'_j = S^o half step, E'_j = S^e,
// O''_j = S^o again, and state j + 1 = (E'_j, O''_j).  The transposes then
// run on (E'_j, O'_j), (E_j, O'_j) and (E_j, O_j).
}  // extern "C"

namespace {

// Reverse pass; dL_du0, dsa and dss are host pointers (dev = false) or
// device pointers (dev = true).
int grad_impl(const double* dL_du0, double* dsa, double* dss, bool dev) {
    if (!C.live) return fail(PM_ESTATE, "no context: call pm_init first");
    if (C.ck <= 0) return fail(PM_ESTATE, "no gradient recording: call pm_set_checkpoint(k > 0) before pm_step");
    if (!dL_du0) return fail(PM_EINVAL, "dL_du0 is NULL");
    hipStream_t s = C.stream();
    const size_t SB = C.state_bytes();
    const long long n = C.ncell;
    const long long T = C.rec_steps;
    const int ck = C.ck;
    const long long ps = C.g.pstride;
    const long long SE = (long long)C.V * ps;      // elements of a state
    const long long EH = C.ve * ps;                 // elements of the even half
    const long long OH = SE - EH;                   // elements of the odd half
    const long long region = 2 * OH + EH;           // O', E', O'' of one step
    const int segs = T > 0 ? (int)std::min<long long>(ck, T) : 1;
    const long long pool_elems = 3 * SE + (long long)segs * region;
    void* pool = nullptr;
    double *grad = nullptr, *outg = nullptr, *gpass = nullptr;
    const long long before = C.dev_bytes;
    const bool timing = C.timing;
    auto cleanup = [&]() {
        dfree(pool); dfree(grad); dfree(outg); dfree(gpass);
        C.dev_bytes = before;
        C.timing = timing;
    };
    int rc;
#define TRYG(x)           \
    do {                  \
        rc = (x);         \
        if (rc) {         \
            cleanup();    \
            return rc;    \
        }                 \
    } while (0)
#define HIPG(x)                                                                        \
    do {                                                                               \
        hipError_t e_ = (x);                                                           \
        if (e_ != hipSuccess) {                                                        \
            cleanup();                                                                 \
            return fail(PM_EDEVICE, std::string(#x) + ": " + hipGetErrorString(e_));   \
        }                                                                              \
    } while (0)
    const int np0 = C.wadj[0].npass, np1 = C.wadj[1].npass;
    const size_t gpb = sizeof(double) * pm::kGradRows * (size_t)n;  // one pass of gradient rows
    const size_t pool_bytes = C.esz * (size_t)pool_elems;
    {
        size_t fr = 0, tot = 0;
        HIPCHK(hipMemGetInfo(&fr, &tot));
        const size_t need = pool_bytes + gpb * (size_t)(np0 + np1 + 1) + sizeof(double) * 2 * (size_t)n;
        if (need > fr)
            return fail(PM_ENOMEM, "gradient pass needs " + std::to_string(need) + " bytes, " +
                                       std::to_string(fr) + " free on the device");
    }
    TRYG(dmalloc(&pool, pool_bytes, "adjoint and segment states"));
    TRYG(dmalloc(&gpass, gpb * (size_t)(np0 + np1), "per-pass gradient rows"));
    TRYG(dmalloc(&grad, gpb, "gradient accumulators"));
    TRYG(dmalloc(&outg, sizeof(double) * 2 * (size_t)n, "gradient output"));
    // pool layout (elements): lam [0, SE), w [SE, 2 SE), segment start state
    // [2 SE, 3 SE), then one region per step
    const long long LAM = 0, W = SE, START = 2 * SE;
    auto reg = [&](long long j) { return 3 * SE + j * region; };
    auto Ej = [&](long long j) { return j == 0 ? START : reg(j - 1) + OH; };
    auto Oj = [&](long long j) { return j == 0 ? START + EH : reg(j - 1) + OH + EH; };
    auto O1 = [&](long long j) { return reg(j); };
    auto E1 = [&](long long j) { return reg(j) + OH; };
    auto O2 = [&](long long j) { return reg(j) + OH + EH; };
    HIPG(pm::launch_fill_zero(pool, (long long)(C.esz * (size_t)SE), s));
    HIPG(pm::launch_fill_zero(gpass, (long long)(gpb * (np0 + np1)), s));
    if (!dev) HIPG(hipMemcpyAsync(C.plane64, dL_du0, sizeof(double) * n, hipMemcpyHostToDevice, s));
    HIPG(pm::launch_from_f64(C.prec, dev ? dL_du0 : C.plane64, C.plane(pool, C.L.slot_of[0]), n, s));
    double* gp_par[2] = {gpass, gpass + (size_t)np0 * pm::kGradRows * (size_t)n};
    C.timing = false;
    auto fwd = [&](int p, long long src, long long tin, long long tout) -> hipError_t {
        if (C.win[p].npass == 0) return hipSuccess;  // a parity without moments (N = 0, odd)
        const pm::Aniso an{C.aniso ? C.gl : nullptr, p ? 0.5 * C.dt : C.dt};
        return pm::launch_sweep_win(C.prec, pool, pm::StateOffs{src, tin, tout, 0, 0}, C.tab, C.tabf,
                                    p ? 8 : 0, an, C.win[p], C.g, s);
    };
    // transpose of the substep of parity p whose old state has halves (E, O)
    auto adj = [&](int p, long long E, long long O) -> hipError_t {
        const pm::Aniso an{C.aniso ? C.gl : nullptr, p ? 0.5 * C.dt : C.dt};
        const long long lam_t = LAM + (p ? EH : 0), lam_d = LAM + (p ? 0 : EH);
        const long long w_t = W + (p ? EH : 0);
        if (C.wadj[p].npass > 0) {
            const pm::StateOffs so{p ? E : O, lam_t, lam_t, p ? O : E, w_t};
            hipError_t e = pm::launch_adj_win(C.prec, 0, pool, so, gp_par[p], C.tab, p ? 8 : 0, an,
                                              C.wadj[p], C.g, s);
            if (e != hipSuccess) return e;
        }
        if (C.wadj[1 - p].npass > 0) {
            const pm::StateOffs so{w_t, lam_d, lam_d, 0, 0};
            return pm::launch_adj_win(C.prec, 1, pool, so, nullptr, C.tab, 0, an, C.wadj[1 - p],
                                      C.g, s);
        }
        return hipSuccess;
    };
    const long long nseg = (T + ck - 1) / ck;
    for (long long gseg = nseg - 1; gseg >= 0; --gseg) {
        const long long s0 = gseg * ck, len = std::min<long long>(s0 + ck, T) - s0;
        HIPG(hipMemcpyAsync((char*)pool + C.esz * START, C.ckpts[gseg], SB, hipMemcpyDeviceToDevice, s));
        for (long long j = 0; j < len; ++j) {
            HIPG(fwd(1, Ej(j), Oj(j), O1(j)));
            HIPG(fwd(0, O1(j), Ej(j), E1(j)));
            if (j + 1 < len) HIPG(fwd(1, E1(j), O1(j), O2(j)));
        }
        for (long long j = len - 1; j >= 0; --j) {
            HIPG(adj(1, E1(j), O1(j)));  // the closing odd half step
            HIPG(adj(0, Ej(j), O1(j)));  // the even step
            HIPG(adj(1, Ej(j), Oj(j)));  // the opening odd half step
        }
    }
    HIPG(pm::launch_grad_sum(gpass, np0 + np1, grad, n, s));
    if (dev) {
        HIPG(pm::launch_grad_final(grad, C.tab, C.sig, C.sig + n, dsa, dss, C.g, C.dt, C.aniso, s));
    } else {
        HIPG(pm::launch_grad_final(grad, C.tab, C.sig, C.sig + n, outg, outg + n, C.g, C.dt, C.aniso, s));
        if (dsa) HIPG(hipMemcpyAsync(dsa, outg, sizeof(double) * n, hipMemcpyDeviceToHost, s));
        if (dss) HIPG(hipMemcpyAsync(dss, outg + n, sizeof(double) * n, hipMemcpyDeviceToHost, s));
    }
    // the temporaries are freed below: the queued work must be done first
    HIPG(hipStreamSynchronize(s));
    cleanup();
#undef TRYG
#undef HIPG
    return PM_OK;
}

}  // namespace

extern "C" {

int pm_grad(const double* dL_du0, double* dsa, double* dss) {
    return grad_impl(dL_du0, dsa, dss, false);
}

int pm_grad_dev(const void* dL_du0, void* dsa, void* dss) {
    return grad_impl((const double*)dL_du0, (double*)dsa, (double*)dss, true);
}

long long pm_recording_id(void) { return g_rec_id; }

int pm_total(double* out) {
    if (!C.live) return fail(PM_ESTATE, "no context: call pm_init first");
    if (!out) return fail(PM_EINVAL, "out is NULL");
    hipStream_t s = C.stream();
    HIPCHK(pm::launch_sum(C.prec, C.plane(C.u, C.L.slot_of[0]), C.ncell, C.red, C.npart,
                          C.red + C.npart, s));
    HIPCHK(hipMemcpyAsync(out, C.red + C.npart, sizeof(double), hipMemcpyDeviceToHost, s));
    HIPCHK(hipStreamSynchronize(s));
    return PM_OK;
}

int pm_check(double* max_abs, long long* n_nonfinite) {
    if (!C.live) return fail(PM_ESTATE, "no context: call pm_init first");
    hipStream_t s = C.stream();
    HIPCHK(pm::launch_check(C.prec, C.u, C.V, C.g, C.red, C.redc, C.ncheck, C.red + C.ncheck,
                            C.redc + C.ncheck, s));
    double m = 0;
    unsigned long long k = 0;
    HIPCHK(hipMemcpyAsync(&m, C.red + C.ncheck, sizeof(double), hipMemcpyDeviceToHost, s));
    HIPCHK(hipMemcpyAsync(&k, C.redc + C.ncheck, sizeof(k), hipMemcpyDeviceToHost, s));
    HIPCHK(hipStreamSynchronize(s));
    if (max_abs) *max_abs = m;
    if (n_nonfinite) *n_nonfinite = (long long)k;
    if (k) return fail(PM_ENONFINITE, std::to_string(k) + " non-finite values in the state");
    return PM_OK;
}

int pm_check_noalloc(void* dev_max_abs, void* dev_nonfinite) {
    if (!C.live) return fail(PM_ESTATE, "no context: call pm_init first");
    if (!dev_max_abs || !dev_nonfinite) return fail(PM_EINVAL, "output pointers must not be NULL");
    const int npart = C.ncheck;
    if (npart > pm::scratch_partials())
        return fail(PM_EINVAL, "pm_check_noalloc: " + std::to_string(npart) + " partial results exceed the " +
                                   std::to_string(pm::scratch_partials()) + " of the static scratch");
    // the scratch's device address: looked up on the first call on a device
    // (hipGetSymbolAddress, return code checked), kept per device
    void* scr = nullptr;
    HIPCHK(pm::scratch_device(&scr));
    double* pmax = (double*)scr;
    unsigned long long* pcnt = (unsigned long long*)((char*)scr + sizeof(double) * pm::scratch_partials());
    // every partial is written before it is read: nothing to clear
    HIPCHK(pm::launch_check(C.prec, C.u, C.V, C.g, pmax, pcnt, npart, (double*)dev_max_abs,
                            (unsigned long long*)dev_nonfinite, C.stream()));
    return PM_OK;
}

int pm_bind_stream(void* stream) {
    g_bound = (hipStream_t)stream;
    return PM_OK;
}

int pm_sync(void) {
    if (!C.live) return fail(PM_ESTATE, "no context: call pm_init first");
    HIPCHK(hipStreamSynchronize(C.stream()));
    return PM_OK;
}

int pm_cfl_warning(void) { return C.live ? C.cfl_warn : 0; }

int pm_timing(int on) {
    if (!C.live) return fail(PM_ESTATE, "no context: call pm_init first");
    HIPCHK(hipStreamSynchronize(C.stream()));
    drop_events();
    C.timing = on != 0;
    return PM_OK;
}

int pm_sweep_times(int* n_odd, double* ms_odd, int* n_even, double* ms_even) {
    if (!C.live) return fail(PM_ESTATE, "no context: call pm_init first");
    HIPCHK(hipStreamSynchronize(C.stream()));
    double t[2] = {0, 0};
    for (int p = 0; p < 2; ++p)
        for (auto& pr : C.ev[p]) {
            float ms = 0;
            HIPCHK(hipEventElapsedTime(&ms, pr.first, pr.second));
            t[p] += ms;
        }
    if (n_odd) *n_odd = (int)C.ev[1].size();
    if (ms_odd) *ms_odd = t[1];
    if (n_even) *n_even = (int)C.ev[0].size();
    if (ms_even) *ms_even = t[0];
    return PM_OK;
}

void pm_finalize(void) {
    if (C.live || C.u || C.own) {
        if (C.own || g_bound) (void)hipStreamSynchronize(C.stream());
        release();
    }
}

const char* pm_last_error(void) { return g_err.c_str(); }

int pm_flux_nnz(int N) {
    if (N < 0 || N > PM_N_MAX) return fail(PM_EINVAL, "N must be in [0, 63]");
    return (int)pm::flux_entries(N).size();
}

int pm_flux_entries(int N, int* row, int* col, int* dir, double* value, int cap) {
    if (N < 0 || N > PM_N_MAX) return fail(PM_EINVAL, "N must be in [0, 63]");
    if (cap < 0) return fail(PM_EINVAL, "cap < 0");
    std::vector<pm::FluxEntry> e = pm::flux_entries(N);
    int k = 0;
    for (; k < (int)e.size() && k < cap; ++k) {
        if (row) row[k] = e[k].row;
        if (col) col[k] = e[k].col;
        if (dir) dir[k] = e[k].dir;
        if (value) value[k] = e[k].val;
    }
    return k;
}

int pm_moment_grid(int N, int moment) {
    if (N < 0 || N > PM_N_MAX) return fail(PM_EINVAL, "N must be in [0, 63]");
    if (moment < 0 || moment >= (N + 1) * (N + 1)) return fail(PM_EINVAL, "moment out of range");
    int l, m;
    pm::moment_lm(moment, l, m);
    return pm::grid_bits(l, m);
}

int pm_moment_slot(int N, int moment) {
    if (N < 0 || N > PM_N_MAX) return fail(PM_EINVAL, "N must be in [0, 63]");
    if (moment < 0 || moment >= (N + 1) * (N + 1)) return fail(PM_EINVAL, "moment out of range");
    return pm::make_layout(N).slot_of[moment];
}

long long pm_halo_plan(int N, int nx, int ny, int nz, int parity, int dirs, long long* moment,
                       long long* cell, long long cap) {
    if (N < 0 || N > PM_N_MAX) return fail(PM_EINVAL, "N must be in [0, 63]");
    if (nx < 1 || ny < 1 || nz < 1) return fail(PM_EINVAL, "grid sizes must be >= 1");
    if (parity != 0 && parity != 1) return fail(PM_EINVAL, "parity must be 0 or 1");
    if (dirs < 1 || dirs > 7) return fail(PM_EINVAL, "dirs must be a nonzero mask of bits 1 (x), 2 (y), 4 (z)");
    if (cap < 0) return fail(PM_EINVAL, "cap < 0");
    const pm::Layout L = pm::make_layout(N);
    HaloPlan hp = halo_plan(L, nx, ny, nz, parity);
    hp.hf = halo_masked(hp.hf, dirs);
    const long long total = hp.hf.end[5];
    if (moment || cell) {
        long long k = 0;
        for (int f = 0; f < 6 && k < cap; ++f) {
            if (hp.hf.area[f] == 0) continue;
            const int d = f >> 1, layer = hp.hf.layer[f];
            const long long cnt = hp.hf.slot0[f + 1] - hp.hf.slot0[f];
            for (long long j = 0; j < cnt && k < cap; ++j)
                for (long long a = 0; a < hp.hf.area[f] && k < cap; ++a, ++k) {
                    long long c;
                    if (d == 0)
                        c = layer + (long long)nx * a;
                    else if (d == 1)
                        c = (a % nx) + (long long)nx * (layer + (long long)ny * (a / nx));
                    else
                        c = a + (long long)nx * ny * layer;
                    if (moment) moment[k] = L.moment_of[hp.slots[hp.hf.slot0[f] + j]];
                    if (cell) cell[k] = c;
                }
        }
    }
    return total;
}

namespace {

int halo_move(int parity, int dirs, void* buf, bool unpack) {
    if (!C.live) return fail(PM_ESTATE, "no context: call pm_init first");
    if (parity != 0 && parity != 1) return fail(PM_EINVAL, "parity must be 0 or 1");
    if (dirs < 1 || dirs > 7) return fail(PM_EINVAL, "dirs must be a nonzero mask of bits 1 (x), 2 (y), 4 (z)");
    if (!buf) return fail(PM_EINVAL, "buffer is NULL");
    const pm::HaloFaces hf = halo_masked(C.halo[parity].hf, dirs);
    HIPCHK(pm::launch_halo(C.prec, unpack, C.u, buf, C.halo_slots[parity], hf, C.g, C.stream()));
    return PM_OK;
}

}  // namespace

int pm_halo_pack(int parity, int dirs, void* device_buf) {
    return halo_move(parity, dirs, device_buf, false);
}

int pm_halo_unpack(int parity, int dirs, const void* device_buf) {
    return halo_move(parity, dirs, const_cast<void*>(device_buf), true);
}

long long pm_device_bytes(void) {
    return C.live ? C.base_bytes + (long long)C.ckpts.size() * (long long)C.state_bytes() : 0;
}

}  // extern "C"
