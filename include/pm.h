/*
 * pm.h -- C ABI of libpm, the MI355X implementation of the staggered-grid
 * P_N time step of StaRMAP (Berghoff, Frank, Seibold, "Massively Parallel
 * Stencil Strategies for Radiation Transport Moment Model Simulations",
 * arXiv 2004.02833).
 *
 * What is computed (paper Sec. 2 and 2.1):
 *   moment system  d_t u + M_x d_x u + M_y d_y u + M_z d_z u + C u = q   (eq. (3))
 *   on a periodic box of nx*ny*nz cubic cells of edge dx.  Moment i lives on
 *   one of eight staggered grids; a time step is the Strang composition
 *   S^o_{dt/2} o S^e_{dt} o S^o_{dt/2} (eq. (6)) of exact exponential
 *   substeps (eq. (5)) driven by half-grid centred differences of the dual
 *   grids (eq. (4)).
 *
 * Conventions shared by every call:
 *   - Moments use the canonical index i = l*l + l + m, 0 <= l <= N, |m| <= l,
 *     for real orthonormal spherical harmonics with z as polar axis
 *     (cos(m phi) for m > 0, sin(|m| phi) for m < 0, no Condon-Shortley sign).
 *     V = (N+1)^2 moments.
 *   - Host field arrays are float64 of length nx*ny*nz, element (x, y, z) at
 *     x + nx*(y + ny*z), 0-based.  sigma_a, sigma_s and q are cell-centred.
 *   - Moment i with reflection parities (ox, oy, oz) is stored at its own
 *     staggered points: cell (x, y, z) holds its value at
 *     ((x + 1/2 + ox/2) dx, (y + 1/2 + oy/2) dx, (z + 1/2 + oz/2) dx)
 *     with the box [0, nx dx) x [0, ny dx) x [0, nz dx).  Moment 0 (the
 *     radiative intensity) is on the cell centres (grid G111).
 *   - Medium: coefficient sigma_a for moment 0 and sigma_a + sigma_s for
 *     l >= 1 (isotropic scattering, eq. (2); per-degree coefficients with
 *     pm_set_scattering); q feeds moment 0 only.  On a staggered point the
 *     coefficient is the mean over the 2, 4 or 8 cells sharing the point.
 *   - One global context, not thread-safe.  The library copies every input
 *     and never keeps a caller pointer; it owns all device memory it uses.
 *   - All int-returning calls give PM_OK (0) on success and a negative code
 *     on failure; pm_last_error() then describes the failure.  A failed call
 *     leaves the context as it was unless stated otherwise.
 */
#ifndef PM_H
#define PM_H

#ifdef __cplusplus
extern "C" {
#endif

#define PM_OK 0
#define PM_EINVAL (-1)     /* bad argument                                    */
#define PM_ENOMEM (-2)     /* device or host allocation failed                */
#define PM_EDEVICE (-3)    /* a HIP call failed                               */
#define PM_ESTATE (-4)     /* call not valid in the current state             */
#define PM_ENONFINITE (-5) /* non-finite value found by pm_check              */

#define PM_FP64 0 /* state, accumulation and update in float64                 */
#define PM_FP32 1 /* float32 state and accumulation; update in float64, rounded */
#define PM_BF16 2 /* bfloat16 state (storage probe); float32 accumulation and update */

#define PM_N_MAX 63

/* Storage precision used by the next pm_init (default PM_FP64).  The decay
 * factors exp(-c tau) and tau E(-c tau) are always computed and kept in
 * float64; FP64 and FP32 apply them in float64, the BF16 storage probe
 * rounds them to float32 for its float32 update.
 * Returns PM_EINVAL for an unknown value. */
int pm_set_precision(int precision);

/* Anisotropic scattering for the next pm_init / pm_init_cells (default:
 * isotropic).  The collision coefficient of degree l is
 *     c_l = sigma_a + (1 - g_l) sigma_s,   g_0 = 1,
 * i.e. Sigma_tl = Sigma_a + Sigma_s0 - Sigma_sl with Sigma_sl = g_l sigma_s
 * (Sec. 2, the moment equations: a scattering kernel that depends only on
 * the angle between directions acts on degree l through its l-th Legendre
 * moment).  g[l - 1] holds g_l for l = 1..count; degrees above count use
 * g_l = 0 (the isotropic value, c_l = sigma_a + sigma_s).  Example:
 * Henyey-Greenstein with asymmetry a has g_l = a^l.  count = 0 (g may be
 * NULL) restores isotropic scattering.  On staggered points c_l is the mean
 * over the cells sharing the point, as for isotropic scattering.  When some
 * g_l != 0 (1 <= l <= N) the sweeps form per-degree decay factors (more
 * arithmetic per cell, the same memory traffic); pm_grad then also
 * differentiates through the (1 - g_l) weights.  The library copies g.
 * Errors: PM_EINVAL (count outside [0, PM_N_MAX], a value not finite or
 * outside [-1, 1]); the setting is then unchanged. */
int pm_set_scattering(const double* g, int count);

/* Create the context (replacing a live one): moment order N (0..PM_N_MAX),
 * grid nx, ny, nz >= 1, cell edge dx > 0, time step dt > 0, host arrays
 * sigma_a >= 0, sigma_s >= 0 (finite) and q (NULL means 0).  Builds the flux
 * matrices M_x, M_y, M_z of eq. (3) in closed form, the staggered-grid
 * assignment of Sec. 2.1, and the per-cell decay tables of eq. (5).  The
 * state starts at zero.  dt above the stability limit dx / (sqrt(3) *
 * lambda_max(N)) only sets a warning (pm_cfl_warning): the paper notes that
 * scattering can stabilise larger steps (Sec. 2.1, last paragraph).
 * Errors: PM_EINVAL, PM_ENOMEM, PM_EDEVICE. */
int pm_init(int N, int nx, int ny, int nz, double dx, double dt,
            const double* sigma_a, const double* sigma_s, const double* q);

/* Same for rectangular cells of edges dx x dy x dz (Sec. 2.1: the box is
 * divided into equal cells of size dx x dy x dz).  A d-difference is divided
 * by its own edge; the stability limit becomes
 * 1 / (lambda_max(N) sqrt(1/dx^2 + 1/dy^2 + 1/dz^2)).  pm_init(..., dx, ...)
 * is pm_init_cells(..., dx, dx, dx, ...).  Staggered points sit at
 * ((x + 1/2 + ox/2) dx, (y + 1/2 + oy/2) dy, (z + 1/2 + oz/2) dz). */
int pm_init_cells(int N, int nx, int ny, int nz, double dx, double dy, double dz, double dt,
                  const double* sigma_a, const double* sigma_s, const double* q);

/* Set moment `moment` (canonical index) from a host float64 array at its
 * staggered points (initial data psi(0, x, Omega), Sec. 2, eq. (1)).
 * Rounds to the storage precision.  Clears a gradient recording (it restarts
 * at the new state).  Errors: PM_ESTATE (no context), PM_EINVAL. */
int pm_write(int moment, const double* src);

/* Same with a device pointer to nx*ny*nz float64 values (read on the bound
 * stream).  The caller keeps ownership. */
int pm_write_dev(int moment, const void* device_src);

/* Advance nsteps >= 0 time steps (eq. (6)): odd half step, even full step,
 * odd half step per step (adjacent odd half steps merged, see pm_set_merge),
 * queued on the bound stream without host synchronisation.  When a gradient
 * recording is active the state is checkpointed every k steps
 * (pm_set_checkpoint).  Without a recording and with timing off, a call is
 * only kernel launches on the bound stream (no allocation, no memset, no
 * synchronisation), so it can be captured into a HIP graph and replayed.
 * Errors: PM_ESTATE, PM_EINVAL, PM_EDEVICE, PM_ENOMEM (checkpoint). */
int pm_step(int nsteps);

/* Step schedule used by pm_step (default 1).  With 1, the odd half step
 * that ends a step and the one that starts the next are applied as one odd
 * substep of length dt: both see the same even moments (eq. (4)) and the odd
 * moments have no source, so the two exact solutions of eq. (5) compose to
 * the exact solution over dt.  n steps then take 2n + 1 sweep launches
 * instead of 3n; states at the end of a pm_step call (and at checkpoints)
 * are step-boundary states, equal to the three-sweep schedule up to
 * rounding.  0 runs every step as its three substeps.  PM_EINVAL otherwise. */
int pm_set_merge(int on);

/* Copy moment `moment` to a host float64 array (synchronises the stream).
 * Moment 0 is the physical output (Sec. 2.1).  Errors: PM_ESTATE, PM_EINVAL. */
int pm_read(int moment, double* dst);

/* Same into a device buffer of nx*ny*nz float64 values (queued on the bound
 * stream, no synchronisation). */
int pm_read_dev(int moment, void* device_dst);

/* Start (k > 0) or stop (k = 0) a gradient recording at the current state.
 * While active, pm_step keeps a device copy of the state every k steps; the
 * steps in between are recomputed by pm_grad.  k < 0 gives PM_EINVAL. */
int pm_set_checkpoint(int k);

/* Reverse pass through every step recorded since pm_set_checkpoint (the
 * paper does not treat derivatives; this is the exact transpose of the
 * discrete step).  Input: host dL/du_0 at the final time (nx*ny*nz; the
 * other moments get a zero cotangent).  Output: host dL/dsigma_a and
 * dL/dsigma_s, cell-centred (either may be NULL).  The forward state is left
 * unchanged.  Errors: PM_ESTATE (no recording), PM_EINVAL, PM_ENOMEM,
 * PM_EDEVICE. */
int pm_grad(const double* dL_du0, double* dsigma_a, double* dsigma_s);

/* Same with device pointers: dL_du0 holds nx*ny*nz float64 values on the
 * device; dsigma_a and dsigma_s (either may be NULL) receive nx*ny*nz
 * float64 values on the device.  The caller keeps ownership of all three.
 * The work is queued on the bound stream; the call returns after it has
 * finished (the pass frees its temporaries).  Errors as pm_grad. */
int pm_grad_dev(const void* dL_du0, void* dsigma_a, void* dsigma_s);

/* Identifier of the recorded forward that pm_grad would differentiate: it
 * changes whenever a recording starts or stops (pm_set_checkpoint), is
 * dropped (pm_write, pm_write_dev, pm_init, pm_init_cells, pm_finalize) or
 * is extended (pm_step while recording).  A caller that stores it after its
 * forward can tell whether pm_grad still refers to that forward.  Never
 * fails. */
long long pm_recording_id(void);

/* Float64 sum of moment 0 over all cells (total intensity; conserved when
 * sigma_a = 0 and q = 0).  Synchronises. */
int pm_total(double* sum_u0);

/* Float64 maximum of |u| over all moments and cells, and the number of
 * non-finite values.  Returns PM_ENONFINITE when that number is not zero. */
int pm_check(double* max_abs, long long* n_nonfinite);

/* For callers that cannot allocate device memory (code under HIP graph
 * capture, tight stepping loops, harnesses that forbid hipMalloc): pm_check
 * without allocation or host synchronisation.  The per-block partial
 * results live in the library's static device scratch (room for 1024
 * partials per GPU, held until the process ends; this call uses all 1024,
 * as pm_check does, for any grid size: the reduction strides over the
 * state).  Writes the float64
 * maximum of |u| over all moments and cells to *dev_max_abs and the number
 * of non-finite values (unsigned 64-bit) to *dev_nonfinite, both device
 * pointers owned by the caller, queued on the bound stream with kernels
 * only (no memset, no allocation, no copy), so it can be captured into a
 * HIP graph.  Every call on a GPU shares that GPU's scratch: calls that
 * overlap on one GPU (other streams, other threads) race.  Errors:
 * PM_ESTATE (no context), PM_EINVAL (NULL output), PM_EDEVICE. */
int pm_check_noalloc(void* dev_max_abs, void* dev_nonfinite);

/* Queue all further work on this hipStream_t (NULL: the library's own
 * stream).  The stream must outlive the context or the next bind. */
int pm_bind_stream(void* hip_stream);

/* Block until all queued work on the bound stream is done. */
int pm_sync(void);

/* 1 if the time step of the live context exceeds the stability limit. */
int pm_cfl_warning(void);

/* Per-sweep timing: when on, pm_step brackets every sweep launch with HIP
 * events on the bound stream.  pm_sweep_times returns the number of odd and
 * even sweep launches and their summed durations in milliseconds since the
 * last reset (synchronises).  pm_timing(0) resets and stops. */
int pm_timing(int on);
int pm_sweep_times(int* n_odd, double* ms_odd, int* n_even, double* ms_even);

/* Release all device memory and the context.  Safe to call twice. */
void pm_finalize(void);

/* Text of the last error (static storage, never NULL). */
const char* pm_last_error(void);

/* ---- host-only queries (no device needed) -------------------------------
 * The closed-form flux matrices and the grid assignment that pm_init uses. */

/* Number of stored nonzeros of M_x + M_y + M_z for order N (<0: error). */
int pm_flux_nnz(int N);

/* Fill up to `cap` entries: target row, source column, direction
 * (0 = x, 1 = y, 2 = z) and value of M_d (not divided by dx).  Returns the
 * number written or PM_EINVAL. */
int pm_flux_entries(int N, int* row, int* col, int* dir, double* value, int cap);

/* Grid of moment i for order N as its parity bits ox | oy << 1 | oz << 2
 * (0 = G111, 1 = G211, 2 = G121, 4 = G112, ...).  <0 on error. */
int pm_moment_grid(int N, int moment);

/* Storage slot of moment i: moments are grouped by grid in the order
 * G111, G221, G212, G122, G211, G121, G112, G222 (Sec. 3.2, reordered
 * components), each grid's moments in increasing canonical index. */
int pm_moment_slot(int N, int moment);

/* ---- halo faces of a split box (one GPU's share) ------------------------
 * When the periodic box is split across GPUs, a sweep of parity p (p = 1:
 * the odd sweep, whose targets have odd l) reads every dual moment (parity
 * 1 - p) at one neighbour per direction d: forward (c + e_d) when the moment
 * is unstaggered in d, backward when it is staggered in d (Sec. 2.1, the
 * half-grid centred differences).  A neighbouring GPU therefore needs only
 * half of the moments on each face (Sec. 3.2 exchanges all of them): the
 * -d neighbour needs this box's layer 0 of the dual moments unstaggered in
 * d (face d-), the +d neighbour its last layer of those staggered in d
 * (face d+).  `dirs` selects the directions the box is split in (bit 0:
 * x, bit 1: y, bit 2: z; 1..7): only their faces are packed.  The packed
 * order is faces x-, x+, y-, y+, z-, z+ (those selected); within a face the
 * moments by storage slot (pm_moment_slot), then the face cells with the two
 * other coordinates in memory order (x fastest).  With x fastest in memory
 * an x face holds one value per row, so splitting only y and z (dirs = 6)
 * keeps every face access a contiguous row or plane.
 *
 * Host query, no device needed: the number of packed elements for order N,
 * an nx x ny x nz box, a sweep of `parity` and the split directions `dirs`;
 * when moment or cell is not NULL, element k's canonical moment and cell
 * x + nx*(y + ny*z) are written for k < cap.  Returns the count, or
 * PM_EINVAL. */
long long pm_halo_plan(int N, int nx, int ny, int nz, int parity, int dirs, long long* moment,
                       long long* cell, long long cap);

/* Gather the halo faces (directions `dirs`) of the live context's state for
 * a sweep of `parity` into a device buffer of pm_halo_plan(...) elements of
 * the storage type (8, 4 or 2 bytes each), queued on the bound stream.  The
 * caller owns the buffer.  Errors: PM_ESTATE, PM_EINVAL. */
int pm_halo_pack(int parity, int dirs, void* device_buf);

/* The inverse scatter: write the packed elements into the same moments and
 * cells of the state (where a neighbouring GPU's faces would land in its
 * ghost layers).  Queued on the bound stream.  Errors: PM_ESTATE, PM_EINVAL. */
int pm_halo_unpack(int parity, int dirs, const void* device_buf);

/* Bytes of device memory the context holds (0 without a context). */
long long pm_device_bytes(void);

#ifdef __cplusplus
}
#endif
#endif /* PM_H */
