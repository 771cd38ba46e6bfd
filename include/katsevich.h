/*
 * katsevich.h -- C ABI of the MI355X (gfx950) pitch-by-pitch Katsevich helical FBP library.
 *
 * The library reconstructs f(x) from a helical cone-beam sinogram g(lambda, alpha, w) measured
 * on a curved detector, following the implementation of Katsevich's inversion formula in
 * Sec. II of "A three-dimensional dual-domain deep network for high-pitch and sparse helical
 * CT reconstruction" (Wang et al., arXiv 2201.02309):
 *   derivative at constant direction (eq. Deriv) -> length-correction weighting (eq. LW) ->
 *   forward height rebinning onto kappa-lines (eqs. FR, w_k) -> Hilbert transform in alpha
 *   (eq. HF with the kernel of eq. e4) -> backward height rebinning (eq. BR) -> post-cosine
 *   weighting (eq. PW) -> backprojection over the PI interval with v*, alpha*, w*
 *   (backprojection step of Sec. II),
 * run pitch by pitch with the per-pitch parameters (kappa-rebinning tables, PI limits,
 * interpolation weights) computed once on the host in float64 and reused for every pitch
 * (Sec. II periodicity relations and the pre-calculating / reconstruction steps).
 *
 * Conventions (all lengths in mm, angles in radians):
 *   helix      a(lambda) = (R cos(lambda+lambda0), R sin(lambda+lambda0), z0 + P lambda/(2 pi)),
 *              P = feed_per_turn (Sec. II helix equation);
 *   views      view n (0 <= n < n_views) at lambda_n = lambda_first + n * 2 pi / views_per_turn;
 *   detector   curved, radius D about the source; column c at fan angle
 *              alpha_c = (c - (det_cols-1)/2 + col_offset) * dalpha, row r at height
 *              w_r = (r - (det_rows-1)/2 + row_offset) * dw (Sec. III-C detector coordinates);
 *   sinogram   float32 [n_views][det_rows][det_cols], columns fastest;
 *   volume     voxel (ix,iy,iz) at (x_first+ix*dx, y_first+iy*dy, z_first+iz*dz),
 *              float32 [nz][ny][nx], x fastest.
 * Slices repeat every pitch when dz divides P (slices_per_pitch = P/dz); otherwise the
 * whole grid is one pitch and no table is reused.
 *
 * Ownership: the caller allocates every device buffer (tables, sinogram, volume,
 * workspace) and passes raw device pointers and a hipStream_t (as void*; NULL = the
 * default stream).  The library never allocates device memory and, except in
 * katsevich_plan_bind, never synchronises the host: compute calls only enqueue kernels on
 * the given stream.  A plan is immutable after katsevich_plan_bind; concurrent compute calls
 * with one bound plan on different streams are safe when their workspaces differ.
 *
 * Errors: every int-returning call returns KATS_OK (0) or a negative status; the detail
 * of the last failure of the calling thread is in katsevich_last_error().  Nothing throws
 * across the ABI.
 */
#ifndef KATSEVICH_H
#define KATSEVICH_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

enum {
    KATS_OK = 0,
    KATS_EINVAL = -1,            /* a null pointer or an out-of-range argument */
    KATS_EINVAL_GEOMETRY = -2,   /* geometry / grid rejected (see katsevich_last_error) */
    KATS_ESHAPE = -3,            /* a buffer size does not match the plan */
    KATS_EWORKSPACE = -4,        /* workspace smaller than katsevich_plan_info says */
    KATS_ENOTBOUND = -5,         /* compute call on a plan without device tables */
    KATS_EHIP = -6,              /* a HIP runtime call or kernel launch failed */
    KATS_ENOMEM = -7             /* host allocation failed while planning */
};

/* Scan geometry (Sec. II helix, Sec. III-C detector coordinates).  R: source radius;
 * D: source-to-detector distance (radius of the curved detector); feed_per_turn: table
 * feed P per turn (the pitch); lambda0, z0: helix start angle / height; lambda_first:
 * lambda of view 0; dalpha, dw: detector column (radians) and row (mm) spacing;
 * col_offset, row_offset: detector offsets in cells; n_views: acquired views;
 * views_per_turn: views per 2 pi (an integer, so views repeat every turn). */
typedef struct katsevich_geometry {
    double R, D, feed_per_turn, lambda0, z0, lambda_first;
    double dalpha, col_offset, dw, row_offset;
    int64_t n_views;
    int32_t views_per_turn, det_cols, det_rows, reserved;
} katsevich_geometry;

/* Voxel grid, see the volume convention above. */
typedef struct katsevich_grid {
    double dx, dy, dz, x_first, y_first, z_first;
    int32_t nx, ny, nz, reserved;
} katsevich_grid;

/* Plan options.  n_psi: number of kappa-lines sampled uniformly on
 * [-pi/2-alpha_m, pi/2+alpha_m] (eq. FR range; 0 -> 2*det_rows+1; must be >= 3);
 * n_threads: host threads used to build the plan (0 -> all hardware threads);
 * flags: KATS_FLAG_HALF_SAMPLE_DERIVATIVE | KATS_FLAG_DETERMINISTIC_ADJOINT (other bits
 * are rejected);
 * bp_slices: slices per backprojection register run (0 -> 16, else 8, 16 or 32; a
 * performance knob, results agree to rounding). */
typedef struct katsevich_options {
    int32_t n_psi, n_threads, flags, bp_slices, hilbert_mode;
} katsevich_options;

/* hilbert_mode: how the Hilbert filter (eq. HF) of katsevich_filter / katsevich_recon runs.
 * KATS_HILBERT_AUTO (0) picks KATS_HILBERT_MFMA; KATS_HILBERT_FFT (1): zero-padded linear
 * convolution by register FFTs (float32); KATS_HILBERT_MFMA (2): the same convolution as a
 * dense Toeplitz product on the matrix cores (even and odd output columns from the odd and
 * even inputs, float32 operands split into float16 pairs with power-of-two range scaling per
 * group of kappa rows, float32 accumulation, the forward rebinning as a pass of its own;
 * agrees with the FFT to ~2.5e-7 relative).  The adjoint (katsevich_recon_backward) always
 * uses the FFT.  Other values: KATS_EINVAL_GEOMETRY. */
#define KATS_HILBERT_AUTO 0
#define KATS_HILBERT_FFT 1
#define KATS_HILBERT_MFMA 2

/* Derivative at constant direction (eq. Deriv) taken at the centre of every 2 x 2 cell of
 * (lambda, alpha) samples instead of by central differences at the samples: each partial
 * derivative is the mean of the two forward differences across the cell.  The filtered
 * data then live on the cell centres, views at lambda_{n+1/2} (n < n_views-1) and columns
 * at alpha_{c+1/2} (c < det_cols-1), and every later step runs on that grid; the sinogram
 * and volume buffers keep their shapes.  Needs n_views >= 4 and det_cols >= 3. */
#define KATS_FLAG_HALF_SAMPLE_DERIVATIVE 1

/* Deterministic adjoint: katsevich_recon_backward accumulates the transposed
 * backprojection in 64-bit fixed point (integer sums do not depend on the order of the
 * atomics) with a power-of-two scale chosen per call from max |d_grad_vol| so that no sum
 * can overflow, then rounds each filtered-data cotangent once to float32: the same bits on
 * every run (the default accumulates in float64 / float32 atomics, equal to rounding but
 * not bit-reproducible).  Costs a larger workspace (workspace_bytes includes it) and
 * time; the forward is unchanged. */
#define KATS_FLAG_DETERMINISTIC_ADJOINT 2

typedef struct katsevich_plan_s *katsevich_plan_t;

/* Sizes and counts of a plan. */
typedef struct katsevich_plan_info {
    uint64_t table_bytes;              /* device table buffer for katsevich_plan_bind */
    uint64_t workspace_bytes;          /* workspace of katsevich_recon */
    uint64_t filtered_bytes;           /* g^F buffer of katsevich_filter / _backproject */
    uint64_t workspace_bytes_filter;   /* workspace of katsevich_filter */
    int64_t first_view, last_view;     /* views filtered: those any valid voxel uses */
    int64_t n_vv;                      /* (voxel, view) pairs with non-zero PI coverage */
    int64_t n_valid_voxels;            /* voxels reconstructed (others are written 0) */
    int32_t n_pitches, slices_per_pitch, n_table_slices, n_psi;
    int32_t window_views;              /* views of one pitch's lambda window W */
    int32_t window_lo;                 /* first window view of pitch 0 (may be < 0) */
    int32_t fft_len, commensurate;     /* Hilbert FFT length; 1 if dz divides P */
    int32_t gf_rows, gf_cols;          /* padded g^F view of katsevich_filter (see below) */
    int32_t atan_degree;               /* degree in t^2 of the backprojector's atan polynomial
                                          (-1: library atan2f) */
    int32_t bp_slices;                 /* slices per backprojection register run */
    int32_t bp_box_rows, bp_box_cols;  /* largest detector footprint box of a backprojection
                                          tile; boxes up to 32 x 64 are staged in LDS, a plan
                                          with larger ones uses the kernel with an HBM path */
    int32_t half_sample;               /* 1 with KATS_FLAG_HALF_SAMPLE_DERIVATIVE: first_view,
                                          last_view, window_lo and the g^F views then count
                                          the cell-centre views lambda_{n+1/2}, and g^F has
                                          det_cols-1 columns */
    int32_t hilbert_mode;              /* the Hilbert path the plan runs: KATS_HILBERT_FFT or
                                          KATS_HILBERT_MFMA */
} katsevich_plan_info;

/* Table ids for katsevich_plan_export (host copies, for tests). */
enum {
    KATS_TABLE_FR_ROW = 1,     /* int32  [n_psi][cols]  floor of the row coordinate of w_kappa */
    KATS_TABLE_FR_WEIGHT = 2,  /* double [n_psi][cols]  its fractional part */
    KATS_TABLE_BR_KAPPA = 3,   /* int32  [rows][cols]   kappa index k0 of psi_hat (<= n_psi-2) */
    KATS_TABLE_BR_WEIGHT = 4,  /* double [rows][cols]   interpolation weight toward k0+1 */
    KATS_TABLE_PSI_HAT = 5,    /* double [rows][cols]   psi_hat(alpha_c, w_r) */
    KATS_TABLE_PI_LI = 6,      /* double [n_table_slices][ny][nx] lambda_i in view units (pitch 0) */
    KATS_TABLE_PI_LO = 7,      /* double [n_table_slices][ny][nx] lambda_o in view units (pitch 0) */
    KATS_TABLE_PI_NFIRST = 8,  /* int32  [n_table_slices][ny][nx] first view with coverage > 0 */
    KATS_TABLE_PI_NLAST = 9,   /* int32  [n_table_slices][ny][nx] last view with coverage > 0 */
    KATS_TABLE_FOV = 10,       /* uint8  [n_table_slices][ny][nx] inside the field of view */
    KATS_TABLE_VALID = 11      /* uint8  [nz][ny][nx] voxel reconstructed (else written 0) */
};

/* Build a plan on the host in float64: validates the geometry (rows must cover the
 * Tam-Danielsson window w_bot(alpha) <= w <= w_top(alpha) over every column, |alpha| <
 * pi/2, positive sizes), computes the kappa-line forward-rebinning table (eqs. FR, w_k),
 * psi_hat and the backward-rebinning table (eq. BR; root of smallest |psi| on the
 * monotone branch), the PI-line limits of every voxel of the first pitch (pre-calculating
 * step 2), the pitch window (eq. maxvalue), the per-view trigonometry and the Hilbert
 * kernel spectrum.  *out receives a new plan to be freed with katsevich_plan_destroy.
 * opts may be NULL (defaults).  Errors: KATS_EINVAL, KATS_EINVAL_GEOMETRY, KATS_ENOMEM. */
int katsevich_plan(const katsevich_geometry *geom, const katsevich_grid *grid,
                   const katsevich_options *opts, katsevich_plan_t *out);

/* Buffers of katsevich_plan_device for a geometry, grid and options.  scratch_bytes: device
 * scratch, free again when the call returns; on return it holds the table pitch's PI
 * tables (each [n_table_slices][ny][nx]): float64 lambda_i and lambda_o in view units at
 * pi_li_offset / pi_lo_offset, int32 first / last covered view at pi_nfirst_offset /
 * pi_nlast_offset, uint8 field-of-view flags at fov_offset.  table_bytes: the device table
 * buffer, laid out for an upper bound of the pitch window (it may exceed the table_bytes
 * of the same plan built on the host). */
typedef struct katsevich_device_plan_sizes {
    uint64_t scratch_bytes, table_bytes;
    uint64_t pi_li_offset, pi_lo_offset, pi_nfirst_offset, pi_nlast_offset, fov_offset;
    int32_t n_table_slices, reserved;
} katsevich_device_plan_sizes;

/* Errors: KATS_EINVAL, KATS_EINVAL_GEOMETRY (as katsevich_plan's validation). */
int katsevich_plan_device_sizes(const katsevich_geometry *geom, const katsevich_grid *grid,
                                const katsevich_options *opts, katsevich_device_plan_sizes *out);

/* The plan of katsevich_plan built on the GPU in float64 (pre-calculating step of Sec. II),
 * every table written by kernels straight into the caller's table buffer d_tables (>=
 * table_bytes of katsevich_plan_device_sizes, 256-byte aligned), to which the returned plan
 * is bound (katsevich_plan_bind then moves the tables device to device).  The rebinning
 * tables, psi_hat, the Hilbert spectrum, the per-view trigonometry and the footprint boxes
 * follow the host builder's float64 arithmetic term for term; the PI lines are solved per
 * voxel by Newton's method on the chord's angle, projected onto [-pi, pi] at every step,
 * safeguarded by bisection (the lines of pre-calculating step 2).  Integer tables equal
 * the host plan's; float tables agree to the last bits of the libm functions.  d_scratch:
 * scratch_bytes, 256-byte aligned.  Enqueued on stream, which the call synchronises once
 * at the end to read back the plan's counts.  Errors as katsevich_plan, plus
 * KATS_EWORKSPACE (scratch too small), KATS_ESHAPE (table buffer too small), KATS_EHIP. */
int katsevich_plan_device(const katsevich_geometry *geom, const katsevich_grid *grid,
                          const katsevich_options *opts, void *d_scratch, uint64_t scratch_bytes,
                          void *d_tables, uint64_t table_bytes, void *stream, katsevich_plan_t *out);

/* Sizes and counts of the plan. */
int katsevich_plan_query(katsevich_plan_t plan, katsevich_plan_info *out);

/* Copy the plan's device tables (table_bytes bytes) into caller-owned device memory
 * d_tables (256-byte aligned) on stream, then wait for that copy.  The buffer must stay
 * alive and unchanged while the plan is used.  May be called again to rebind (a plan built
 * by katsevich_plan_device copies from the buffer it is bound to; binding that same buffer
 * again does nothing). */
int katsevich_plan_bind(katsevich_plan_t plan, void *d_tables, uint64_t bytes, void *stream);

/* Copy one host table (KATS_TABLE_*) into host_dst of exactly the table's size in bytes
 * (KATS_ESHAPE otherwise).  Used by tests to compare integer tables bit for bit.  A plan
 * built by katsevich_plan_device exports the rebinning tables and the validity mask (read
 * back from its device PI table); its PI tables themselves are KATS_EINVAL here (they are
 * in the scratch of the build on return). */
int katsevich_plan_export(katsevich_plan_t plan, int which, void *host_dst, uint64_t bytes);

/* Reconstruct: d_sino float32 [n_views][rows][cols] -> d_vol float32 [nz][ny][nx].
 * Invalid voxels are written 0.  d_ws: device workspace of at least workspace_bytes
 * (256-byte aligned).  Asynchronous on stream.  Errors: KATS_EINVAL, KATS_ENOTBOUND,
 * KATS_EWORKSPACE, KATS_EHIP. */
int katsevich_recon(katsevich_plan_t plan, const float *d_sino, float *d_vol,
                    void *d_ws, uint64_t ws_bytes, void *stream);

/* Filtering stage alone (eqs. Deriv, LW, FR, HF, BR, PW): d_sino -> d_gF float32
 * [last_view-first_view+1][gf_rows][gf_cols] (filtered_bytes) holding g^F of views
 * first_view..last_view with a zero border: gf_rows = rows + 2*KATS_GF_PAD, gf_cols =
 * cols + 2*KATS_GF_PAD rounded up to a multiple of 4, element [v][r+KATS_GF_PAD][c+KATS_GF_PAD]
 * is detector cell (r, c) and every other element is 0.
 * d_ws: at least workspace_bytes_filter.  Asynchronous on stream.  Errors: KATS_EINVAL,
 * KATS_ENOTBOUND, KATS_EWORKSPACE, KATS_EHIP. */
#define KATS_GF_PAD 2
int katsevich_filter(katsevich_plan_t plan, const float *d_sino, float *d_gF,
                     void *d_ws, uint64_t ws_bytes, void *stream);

/* Backprojection stage alone (backprojection step of Sec. II, every pitch reusing the
 * first pitch's tables): d_gF as written by katsevich_filter -> d_vol.  Asynchronous.
 * Errors: KATS_EINVAL, KATS_ENOTBOUND, KATS_EHIP. */
int katsevich_backproject(katsevich_plan_t plan, const float *d_gF, float *d_vol, void *stream);

/* Grouped backprojection of n reconstructions (serving): item i backprojects d_gF[i]
 * (katsevich_filter output of plans[i]) into d_vol[i], exactly as katsevich_backproject
 * would (bit-identical results).  One launch covers the (pitch, slice run, tile) tasks of
 * up to 16 items, so reconstructions of different sizes, pitches and grids fill the GPU
 * together; items whose footprint boxes all fit the kernel's LDS tile are grouped apart
 * from the others (see bp_box_rows / bp_box_cols of katsevich_plan_info).  All plans
 * must be bound and use the same bp_slices.  No device memory besides the arrays named;
 * the host arrays may be reused when the call returns.  Asynchronous on stream.
 * Errors: KATS_EINVAL, KATS_ENOTBOUND, KATS_EHIP. */
int katsevich_backproject_batch(const katsevich_plan_t *plans, const float *const *d_gF,
                                float *const *d_vol, int n, void *stream);

/* Exact adjoint of katsevich_recon (transpose of the discrete operator): d_grad_vol
 * float32 [nz][ny][nx] -> d_grad_sino float32 [n_views][rows][cols] (overwritten).
 * d_ws: at least workspace_bytes.  Asynchronous on stream.  Errors: KATS_EINVAL,
 * KATS_ENOTBOUND, KATS_EWORKSPACE, KATS_EHIP. */
int katsevich_recon_backward(katsevich_plan_t plan, const float *d_grad_vol, float *d_grad_sino,
                             void *d_ws, uint64_t ws_bytes, void *stream);

/* ---- Sparse-detector data path and image metrics (Sec. III-C data preparation, Sec. IV
 * metrics).  Plan-free, asynchronous on stream, no device allocation; device buffers are
 * the caller's.  Errors: KATS_EINVAL (null pointer, bad size), KATS_EWORKSPACE, KATS_EHIP. */

/* Interpolate a sparse-detector sinogram back to the full column grid: the sparse data
 * hold columns 0, step, 2 step, ... of a detector with cols columns (Sec. III-C keeps every
 * 4th), d_sparse float32 [n_lines][ns] with ns = ceil(cols / step), n_lines = n_views *
 * rows; d_full float32 [n_lines][cols] gets the linear interpolation in alpha between
 * neighbouring kept columns, and the last kept column's value beyond it (at most 2^34
 * output samples).  n_lines = 0 does nothing (the pointers may then be null). */
int katsevich_sparse_upsample(const float *d_sparse, float *d_full, int64_t n_lines, int32_t cols,
                              int32_t step, void *stream);

/* Device scratch (bytes) of katsevich_max and katsevich_rmse_ssim (fixed, 256-byte
 * aligned buffer, any n). */
uint64_t katsevich_data_scratch_bytes(void);

/* d_max[0] = max of the n values of d_x (n >= 1); deterministic. */
int katsevich_max(const float *d_x, uint64_t n, float *d_max, void *d_scratch,
                  uint64_t scratch_bytes, void *stream);

/* Noisy sinogram of Sec. III-C: with M = d_max[0] (the maximum of d_in, e.g. from
 * katsevich_max) each element becomes M log(I0 / counts), counts = lambda + sqrt(lambda) z1
 * + sqrt(var) z2, lambda = I0 exp(-g / M): Poisson photon counts by their normal limit
 * (lambda >= I0 / e here) plus Gaussian electronic noise of mean 0 and variance var,
 * counts below 1 raised to 1.  z1, z2: Box-Muller transform of the 24-bit uniforms
 * u1 = ((a >> 40) + 1) 2^-24, u2 = (b >> 40) 2^-24, where elements 2k and 2k+1 take
 * (a, b) = (x0, x1) and (x2, x3) of the Philox4x64-10 block of counter (k, 0, 0, 0) and
 * key (seed, 0).  The transcendentals are the hardware's single-precision ones.  d_out
 * may equal d_in.  n = 0 does nothing (the pointers may then be null). */
int katsevich_add_noise(const float *d_in, float *d_out, uint64_t n, const float *d_max, double I0,
                        double var, uint64_t seed, void *stream);

/* d_result[0] = RMSE = sqrt(sum (f - ref)^2 / n); d_result[1] = SSIM of the two whole
 * images (one window): (2 mu_f mu_r + c1)(2 cov + c2) / ((mu_f^2 + mu_r^2 + c1)(var_f +
 * var_r + c2)), population moments, c1 = (0.01 (max ref - min ref))^2, c2 = (0.03 (max
 * ref - min ref))^2 (Sec. IV).  Float64 accumulation, two passes, deterministic. */
int katsevich_rmse_ssim(const float *d_f, const float *d_ref, uint64_t n, double *d_result,
                        void *d_scratch, uint64_t scratch_bytes, void *stream);

/* For callers that cannot allocate device memory (code under HIP graph capture, tight
 * serving loops, harnesses that forbid hipMalloc): katsevich_rmse_ssim with the same
 * kernels and result, its reduction partials kept in a library-owned static device array
 * of KATS_STATIC_SCRATCH_BYTES instead of a caller scratch buffer.  Each GPU holds its own
 * copy of the array until the process ends; its address is looked up on the first call
 * on a device (with that device current), and the call allocates nothing.  The reduction
 * needs the same fixed scratch for any n, so no n >= 1 is too large; a library whose
 * static array were smaller than that need would return KATS_EWORKSPACE.  Nothing in the
 * array needs clearing (every launch writes the partials it reads), but every call on one
 * GPU shares it: calls that overlap on one GPU (other streams, other threads) race and
 * must be serialised by the caller.  Errors: KATS_EINVAL (null pointer, n < 1),
 * KATS_EWORKSPACE, KATS_EHIP. */
#define KATS_STATIC_SCRATCH_BYTES 164096
int katsevich_rmse_ssim_noscratch(const float *d_f, const float *d_ref, uint64_t n, double *d_result,
                                  void *stream);

/* Free a plan (NULL is ignored).  Device buffers stay with the caller. */
void katsevich_plan_destroy(katsevich_plan_t plan);

/* Static description of a status code; never NULL. */
const char *katsevich_status_string(int status);

/* Detail of the calling thread's last error ("" if none); valid until its next call. */
const char *katsevich_last_error(void);

#ifdef __cplusplus
}
#endif

#endif /* KATSEVICH_H */
