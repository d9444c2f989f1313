/*
 * FP64 CPU oracle for the staggered-grid P_N step -- TEST INFRASTRUCTURE ONLY.
 * Called through ctypes by the test suite and by the CPU-baseline leg of the
 * benchmark; the product library never links or calls it.
 *
 * It is the same literal scheme as oracle/stepper.py written as plain loops,
 * for configurations too large for numpy (Berghoff, Frank, Seibold,
 * arXiv 2004.02833, Sec. 2.1):
 *   - moment i sits on G_{1+ox,1+oy,1+oz}; 0-based cell c holds it at
 *     (c + 1/2 + o/2) h in every direction;
 *   - half-grid difference: target staggered in d -> (u[c+e_d] - u[c]) / h_d,
 *     otherwise (u[c] - u[c-e_d]) / h_d, periodic wrap;
 *   - eq. (4): r_i = q_i - sum_d sum_j M_d[i,j] D_d u_j from the dual parity;
 *   - eq. (5): u_i <- u_i + tau (r_i - c_i u_i) E(-c_i tau), E(z) = expm1(z)/z,
 *     E(0) = 1;
 *   - eq. (6): odd half step, even full step, odd half step.
 * c = sigma_a for moment 0 and sigma_a + sigma_s otherwise, averaged over the
 * cells that share a staggered point; q acts on moment 0 only.  With
 * anisotropic scattering (per-degree moments g_l of a phase function, g_0 = 1)
 * moment i of degree l >= 1 uses c = sigma_a + (1 - g_l) sigma_s instead,
 * averaged the same way; its field is formed per moment when it is updated.
 *
 * The flux matrices and the parities come in as arguments (the Python oracle
 * computes them by quadrature and by evaluating reflections).
 *
 * Adjoint (paper silent; chain rule of the same scheme): see pno_grad.
 */
#include <math.h>
#include <stdlib.h>
#include <string.h>
#include <stdint.h>
#ifdef _OPENMP
#include <omp.h>
#endif

typedef struct {
    int V, nx, ny, nz;
    long ncell;
    double h[3], dt;
    const int *o;            /* V*3 parities */
    /* CSR by target row */
    int *rp, *cj, *cd;
    double *cv;
    const double *q;
    double *cbar[9];         /* coefficient set k: 0..7 family, 8 = moment 0 */
    double *Eodd[9], *Eeven[9];
    const double *sa, *ss;
    const double *gl;        /* NULL (isotropic) or g_0..g_N */
    int *deg;                /* degree l of moment i */
    double *work;            /* one coefficient field (anisotropic case) */
} prob_t;

static int fam_of(const int *o) { return o[0] + 2 * o[1] + 4 * o[2]; }
static int cset(const prob_t *P, int i) { return i == 0 ? 8 : fam_of(P->o + 3 * i); }

static double Efun(double z) { return z == 0.0 ? 1.0 : expm1(z) / z; }

static long cell(const prob_t *P, int x, int y, int z) {
    return (long)x + (long)P->nx * ((long)y + (long)P->ny * z);
}

static int wrap(int a, int n) { a %= n; return a < 0 ? a + n : a; }

/* mean of field f over the 2^|o| cells sharing the staggered point of cell c */
static void stagger_mean(const prob_t *P, const double *f, const int *o, double *out) {
#pragma omp parallel for schedule(static)
    for (int z = 0; z < P->nz; ++z)
        for (int y = 0; y < P->ny; ++y)
            for (int x = 0; x < P->nx; ++x) {
                double s = 0.0; int n = 0;
                for (int bz = 0; bz <= o[2]; ++bz)
                    for (int by = 0; by <= o[1]; ++by)
                        for (int bx = 0; bx <= o[0]; ++bx) {
                            s += f[cell(P, wrap(x + bx, P->nx), wrap(y + by, P->ny), wrap(z + bz, P->nz))];
                            ++n;
                        }
                out[cell(P, x, y, z)] = s / n;
            }
}

static int setup(prob_t *P, int V, int nx, int ny, int nz, double hx, double hy, double hz,
                 double dt, const int *o, int nnz, const int *ti, const int *sj, const int *dir,
                 const double *val, const double *sa, const double *ss, const double *q,
                 const double *gl) {
    memset(P, 0, sizeof *P);
    P->V = V; P->nx = nx; P->ny = ny; P->nz = nz;
    P->ncell = (long)nx * ny * nz;
    P->h[0] = hx; P->h[1] = hy; P->h[2] = hz; P->dt = dt;
    P->o = o; P->q = q; P->sa = sa; P->ss = ss; P->gl = gl;
    if (V <= 0 || nx <= 0 || ny <= 0 || nz <= 0) return -1;
    P->deg = malloc(sizeof(int) * V);
    for (int i = 0, l = 0; i < V; ++i) {
        while ((l + 1) * (l + 1) <= i) ++l;
        P->deg[i] = l;
    }
    P->work = gl ? malloc(sizeof(double) * P->ncell) : NULL;
    P->rp = calloc((size_t)V + 1, sizeof(int));
    P->cj = malloc(sizeof(int) * (nnz > 0 ? nnz : 1));
    P->cd = malloc(sizeof(int) * (nnz > 0 ? nnz : 1));
    P->cv = malloc(sizeof(double) * (nnz > 0 ? nnz : 1));
    for (int k = 0; k < nnz; ++k) P->rp[ti[k] + 1]++;
    for (int i = 0; i < V; ++i) P->rp[i + 1] += P->rp[i];
    int *fill = calloc((size_t)V, sizeof(int));
    for (int k = 0; k < nnz; ++k) {
        int pos = P->rp[ti[k]] + fill[ti[k]]++;
        P->cj[pos] = sj[k]; P->cd[pos] = dir[k]; P->cv[pos] = val[k];
    }
    free(fill);
    double *tot = malloc(sizeof(double) * P->ncell);
    for (long c = 0; c < P->ncell; ++c) tot[c] = sa[c] + ss[c];
    for (int k = 0; k < 9; ++k) {
        int ok[3];
        if (k == 8) { ok[0] = ok[1] = ok[2] = 0; }
        else { ok[0] = k & 1; ok[1] = (k >> 1) & 1; ok[2] = (k >> 2) & 1; }
        P->cbar[k] = malloc(sizeof(double) * P->ncell);
        P->Eodd[k] = malloc(sizeof(double) * P->ncell);
        P->Eeven[k] = malloc(sizeof(double) * P->ncell);
        stagger_mean(P, k == 8 ? sa : tot, ok, P->cbar[k]);
        for (long c = 0; c < P->ncell; ++c) {
            P->Eodd[k][c] = Efun(-P->cbar[k][c] * 0.5 * dt);
            P->Eeven[k][c] = Efun(-P->cbar[k][c] * dt);
        }
    }
    free(tot);
    return 0;
}

static void teardown(prob_t *P) {
    free(P->rp); free(P->cj); free(P->cd); free(P->cv);
    for (int k = 0; k < 9; ++k) { free(P->cbar[k]); free(P->Eodd[k]); free(P->Eeven[k]); }
    free(P->deg); free(P->work);
}

/* Coefficient field of moment i on its own points (anisotropic case):
 * the staggered mean of sigma_a + (1 - g_l) sigma_s (sigma_a for i = 0),
 * written to P->work. */
static const double *aniso_cbar(const prob_t *P, int i) {
    double *f = malloc(sizeof(double) * P->ncell);
    const double w = 1.0 - P->gl[P->deg[i]];
    for (long c = 0; c < P->ncell; ++c) f[c] = i == 0 ? P->sa[c] : P->sa[c] + w * P->ss[c];
    stagger_mean(P, f, P->o + 3 * i, P->work);
    free(f);
    return P->work;
}

/* r_i at cell (x,y,z): q_i - sum M_d[i,j] D_d u_j */
static double residual(const prob_t *P, const double *u, int i, int x, int y, int z) {
    const int *oi = P->o + 3 * i;
    long c = cell(P, x, y, z);
    double r = (i == 0 && P->q) ? P->q[c] : 0.0;
    for (int k = P->rp[i]; k < P->rp[i + 1]; ++k) {
        const double *uj = u + (long)P->cj[k] * P->ncell;
        int d = P->cd[k];
        int xs = x, ys = y, zs = z, sgn = oi[d] ? 1 : -1;
        if (d == 0) xs = wrap(x + sgn, P->nx);
        else if (d == 1) ys = wrap(y + sgn, P->ny);
        else zs = wrap(z + sgn, P->nz);
        double nb = uj[cell(P, xs, ys, zs)];
        double D = oi[d] ? (nb - uj[c]) / P->h[d] : (uj[c] - nb) / P->h[d];
        r -= P->cv[k] * D;
    }
    return r;
}

static void substep(const prob_t *P, double *u, int parity, double tau, int even_tau) {
    for (int i = 0; i < P->V; ++i) {
        const int *oi = P->o + 3 * i;
        if (((oi[0] + oi[1] + oi[2]) & 1) != parity) continue;
        int k = cset(P, i);
        const double *cb = P->gl ? aniso_cbar(P, i) : P->cbar[k];
        const double *Ek = P->gl ? NULL : even_tau ? P->Eeven[k] : P->Eodd[k];
        double *ui = u + (long)i * P->ncell;
#pragma omp parallel for schedule(static)
        for (int z = 0; z < P->nz; ++z)
            for (int y = 0; y < P->ny; ++y)
                for (int x = 0; x < P->nx; ++x) {
                    long c = cell(P, x, y, z);
                    double r = residual(P, u, i, x, y, z);
                    double E = Ek ? Ek[c] : Efun(-cb[c] * tau);
                    ui[c] = ui[c] + tau * (r - cb[c] * ui[c]) * E;
                }
    }
}

static void full_step(const prob_t *P, double *u) {
    substep(P, u, 1, 0.5 * P->dt, 0);
    substep(P, u, 0, P->dt, 1);
    substep(P, u, 1, 0.5 * P->dt, 0);
}

/* gl: NULL for isotropic scattering, else g_0..g_N (g_0 = 1). */
int pno_run(int V, int nx, int ny, int nz, double hx, double hy, double hz, double dt,
            const int *o, int nnz, const int *ti, const int *sj, const int *dir, const double *val,
            const double *sa, const double *ss, const double *q, const double *gl, double *u,
            int nsteps, int nthreads) {
#ifdef _OPENMP
    if (nthreads > 0) omp_set_num_threads(nthreads);
#endif
    prob_t P;
    if (setup(&P, V, nx, ny, nz, hx, hy, hz, dt, o, nnz, ti, sj, dir, val, sa, ss, q, gl)) return -1;
    for (int s = 0; s < nsteps; ++s) full_step(&P, u);
    teardown(&P);
    return 0;
}

int pno_threads(void) {
#ifdef _OPENMP
    int n = 0;
#pragma omp parallel
    {
#pragma omp single
        n = omp_get_num_threads();
    }
    return n;
#else
    return 1;
#endif
}

/* ---------------- adjoint ----------------
 * Transpose of one substep with targets i of the given parity:
 *   gc_k  += lam_i (u_i d alpha/dc + r_i d beta/dc)   (k = coefficient set of i;
 *            anisotropic case: k = family of i into the sigma_a sums and,
 *            weighted by 1 - g_l, into the sigma_s sums gc[9 + family])
 *   lam_j += - sum M_d[i,j] D_d^T (beta_i lam_i)      (j dual)
 *   lam_i  = alpha_i lam_i
 * with alpha = exp(-c tau), beta = tau E(-c tau).  D^T of the forward
 * difference (w[c] from w[c-1] - w[c]) and of the backward one (w[c] - w[c+1]).
 */
static double dbeta(double c, double tau) {
    double z = c * tau;
    if (fabs(z) < 1e-3) return tau * tau * (-0.5 + z / 3.0 - z * z / 8.0 + z * z * z / 30.0);
    double a = exp(-z), b = -expm1(-z) / c;
    return (tau * a - b) / c;
}

static void substep_T(const prob_t *P, const double *u_old, double *lam, int parity, double tau,
                      double **gc /* 9 fields per tau kind folded by caller */) {
    long n = P->ncell;
    double *w = malloc(sizeof(double) * n);
    for (int i = 0; i < P->V; ++i) {
        const int *oi = P->o + 3 * i;
        if (((oi[0] + oi[1] + oi[2]) & 1) != parity) continue;
        int k = cset(P, i);
        const double *cb = P->gl ? aniso_cbar(P, i) : P->cbar[k];
        const double *ui = u_old + (long)i * n;
        double *li = lam + (long)i * n;
        double *g = P->gl ? gc[fam_of(oi)] : gc[k];
        double *gs = P->gl ? gc[9 + fam_of(oi)] : NULL;
        const double ws = P->gl ? 1.0 - P->gl[P->deg[i]] : 0.0;
#pragma omp parallel for schedule(static)
        for (int z = 0; z < P->nz; ++z)
            for (int y = 0; y < P->ny; ++y)
                for (int x = 0; x < P->nx; ++x) {
                    long c = cell(P, x, y, z);
                    double cc = cb[c];
                    double a = exp(-cc * tau), b = tau * Efun(-cc * tau);
                    double r = residual(P, u_old, i, x, y, z);
                    double gcv = li[c] * (ui[c] * (-tau * a) + r * dbeta(cc, tau));
                    g[c] += gcv;
                    if (gs && i != 0) gs[c] += ws * gcv;
                    w[c] = b * li[c];
                }
        for (int kk = P->rp[i]; kk < P->rp[i + 1]; ++kk) {
            double *lj = lam + (long)P->cj[kk] * n;
            int d = P->cd[kk];
            double m = P->cv[kk], hd = P->h[d];
            int fwd = oi[d];
#pragma omp parallel for schedule(static)
            for (int z = 0; z < P->nz; ++z)
                for (int y = 0; y < P->ny; ++y)
                    for (int x = 0; x < P->nx; ++x) {
                        int s = fwd ? -1 : 1;
                        int xs = x, ys = y, zs = z;
                        if (d == 0) xs = wrap(x + s, P->nx);
                        else if (d == 1) ys = wrap(y + s, P->ny);
                        else zs = wrap(z + s, P->nz);
                        long c = cell(P, x, y, z), cn = cell(P, xs, ys, zs);
                        double DT = fwd ? (w[cn] - w[c]) / hd : (w[c] - w[cn]) / hd;
                        lj[c] -= m * DT;
                    }
        }
        for (long c = 0; c < n; ++c) li[c] *= exp(-cb[c] * tau);
    }
    free(w);
}

/* L = 1/2 sum (u_0(T) - target)^2 and its gradients w.r.t. sigma_a, sigma_s.
 * Step-start states are checkpointed every ck steps and recomputed per
 * segment; within a step the two intermediate states are recomputed. */
double pno_grad(int V, int nx, int ny, int nz, double hx, double hy, double hz, double dt,
                const int *o, int nnz, const int *ti, const int *sj, const int *dir,
                const double *val, const double *sa, const double *ss, const double *q,
                const double *gl, const double *u0, int nsteps, int ck, const double *target,
                double *dsa, double *dss, int nthreads) {
#ifdef _OPENMP
    if (nthreads > 0) omp_set_num_threads(nthreads);
#endif
    prob_t P;
    if (setup(&P, V, nx, ny, nz, hx, hy, hz, dt, o, nnz, ti, sj, dir, val, sa, ss, q, gl)) return NAN;
    long n = P.ncell, sz = (long)V * n;
    if (ck < 1) ck = 1;
    int nseg = (nsteps + ck - 1) / ck;
    double *cp = malloc(sizeof(double) * sz * (nseg > 0 ? nseg : 1));
    double *u = malloc(sizeof(double) * sz);
    memcpy(u, u0, sizeof(double) * sz);
    for (int s = 0; s < nsteps; ++s) {
        if (s % ck == 0) memcpy(cp + (long)(s / ck) * sz, u, sizeof(double) * sz);
        full_step(&P, u);
    }
    double L = 0.0;
    double *lam = calloc(sz, sizeof(double));
    for (long c = 0; c < n; ++c) { double d = u[c] - target[c]; L += 0.5 * d * d; lam[c] = d; }
    double *gc[17];  /* sets 0..8; anisotropic case: 0..7 sigma_a and 9..16 sigma_s sums */
    for (int k = 0; k < 17; ++k) gc[k] = calloc(n, sizeof(double));
    double *seg = malloc(sizeof(double) * sz * ck);
    double *ua = malloc(sizeof(double) * sz), *ub = malloc(sizeof(double) * sz);
    for (int g = nseg - 1; g >= 0; --g) {
        int s0 = g * ck, s1 = s0 + ck < nsteps ? s0 + ck : nsteps;
        memcpy(seg, cp + (long)g * sz, sizeof(double) * sz);
        for (int s = s0 + 1; s < s1; ++s) {
            memcpy(seg + (long)(s - s0) * sz, seg + (long)(s - s0 - 1) * sz, sizeof(double) * sz);
            full_step(&P, seg + (long)(s - s0) * sz);
        }
        for (int s = s1 - 1; s >= s0; --s) {
            const double *un = seg + (long)(s - s0) * sz;
            memcpy(ua, un, sizeof(double) * sz);
            substep(&P, ua, 1, 0.5 * dt, 0);
            memcpy(ub, ua, sizeof(double) * sz);
            substep(&P, ub, 0, dt, 1);
            substep_T(&P, ub, lam, 1, 0.5 * dt, gc);
            substep_T(&P, ua, lam, 0, dt, gc);
            substep_T(&P, un, lam, 1, 0.5 * dt, gc);
        }
    }
    /* interpolation transpose: c_k(c) = mean of sigma over cells c + b */
    memset(dsa, 0, sizeof(double) * n);
    memset(dss, 0, sizeof(double) * n);
    for (int k = 0; k < 9; ++k) {
        int ok[3];
        if (k == 8) { ok[0] = ok[1] = ok[2] = 0; }
        else { ok[0] = k & 1; ok[1] = (k >> 1) & 1; ok[2] = (k >> 2) & 1; }
        double wgt = 1.0 / (double)((1 + ok[0]) * (1 + ok[1]) * (1 + ok[2]));
        for (int z = 0; z < nz; ++z)
            for (int y = 0; y < ny; ++y)
                for (int x = 0; x < nx; ++x) {
                    long cc = cell(&P, x, y, z);
                    double gv = gc[k][cc] * wgt;
                    double gsv = (gl ? (k < 8 ? gc[9 + k][cc] : 0.0) : (k != 8 ? gc[k][cc] : 0.0)) * wgt;
                    for (int bz = 0; bz <= ok[2]; ++bz)
                        for (int by = 0; by <= ok[1]; ++by)
                            for (int bx = 0; bx <= ok[0]; ++bx) {
                                long t = cell(&P, wrap(x + bx, nx), wrap(y + by, ny), wrap(z + bz, nz));
                                dsa[t] += gv;
                                dss[t] += gsv;
                            }
                }
    }
    for (int k = 0; k < 17; ++k) free(gc[k]);
    free(cp); free(u); free(lam); free(seg); free(ua); free(ub);
    teardown(&P);
    return L;
}
