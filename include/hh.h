/*
 * hh.h — C ABI of the PCA digital-holography hot path on AMD Instinct MI355X (gfx950).
 *
 * Method: Puyo et al., "Real-time digital holography of the retina by principal
 * component analysis" (arXiv:2004.00923).  A stack of n_t consecutive 16-bit
 * inline interferograms becomes one power-Doppler image in five steps:
 *   (a) Fresnel propagation of every frame, Eq. (1): chirp multiply + 2D FFT;
 *   (b) the n_t x n_t time-lagged covariance C = H^{t*} H, Eq. (4);
 *   (c) its eigendecomposition C = V Lambda V^{t*}, Eq. (5);
 *   (d) projection of the stack on the eigenvectors, H_breve = H V I_f, Eq. (6);
 *   (e) the image M(x,y) = sum over kept components of |H_breve|^2, Eq. (7).
 *
 * Conventions shared by every entry point
 * ---------------------------------------
 *  - Array pointers are DEVICE pointers on the current HIP device, owned by the
 *    caller; the library never frees or keeps them.  All arrays are dense,
 *    C-order, without padding.
 *  - Complex arrays are interleaved (re, im): "complex64" = 2 x float,
 *    "complex128" = 2 x double.
 *  - A stack is frame-major [n][ny][nx] (nx is the fast axis); the paper's
 *    space-time matrix H (n_x n_y rows, n_t columns) is its transpose view:
 *    H[p][t] = stack[t][p], p = y * nx + x.
 *  - `stream` is a hipStream_t passed as void* (NULL = the null stream).  Work is
 *    enqueued on it and the call returns without waiting for the device.
 *  - Host-side failures (bad parameters, NULL pointers, a workspace that is too
 *    small, an unsupported size) return synchronously and enqueue nothing.
 *    A failing HIP launch returns HH_E_DEVICE.  The text of the last failure on
 *    the calling thread is in hh_last_error().
 *  - Device tables (chirps, twiddles) are built on the first call for a given
 *    (device, wavelength, distance, pitch, nx, ny) and cached until
 *    hh_plan_cache_clear(); that first call allocates and copies synchronously.
 *  - Entry points never synchronise the host with the device, except that
 *    first-call table build.
 */
#ifndef HH_H
#define HH_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef int32_t hh_status;

enum {
  HH_OK = 0,
  HH_E_INVALID = 1,       /* bad parameter or NULL pointer */
  HH_E_UNSUPPORTED = 2,   /* valid but not implemented (size, precision form) */
  HH_E_WORKSPACE = 3,     /* workspace NULL or smaller than required */
  HH_E_DEVICE = 4,        /* a HIP runtime call or kernel launch failed */
  HH_E_NOT_CONVERGED = 5  /* reserved for host-side reporting of info < 0 */
};

/* Eigensolver of step (c) used by the pipeline entry points (both FP64, both give
 * the eigenpairs of Eq. (5) to rounding; they differ in speed and in what info counts). */
enum {
  HH_EIGH_JACOBI = 0,   /* parallel cyclic Jacobi (hh_eigh) */
  HH_EIGH_TRIDIAG = 1   /* Householder reduction to real tridiagonal form, implicit QL (hh_eigh_tridiag) */
};

/* Arithmetic of the covariance contraction of step (b), Eq. (4), and of the
 * hologram storage.  In every form the stack is split per pixel as
 * H = m 1^T + R (m a per-pixel reference, the temporal mean) and the rank-one
 * terms of C are carried in FP32/FP64; the forms differ in the operands of the
 * R^H R contraction.  Forms 1-5 read the FP32 hologram, so HBM traffic is that
 * of HH_FP32; they trade accuracy for MFMA and register work.  HH_FP16_STORE
 * changes what is stored: step (a) transforms the mean frame once (m, FP32) and
 * each frame minus the mean (R, by linearity of Eq. (1)), and writes R as FP16
 * scaled by s = 1 / (2 nx ny) (|R| <= nx ny 65535, so s R never overflows); the
 * covariance runs on FP16 MFMA straight from R, and the projection of step (d)
 * reads m + R / s.  It halves the hologram traffic and applies only to the
 * entry points that start from frames (hh_pipeline, hh_pipeline_batch,
 * hh_graph_create).  HH_EXACT computes C without the holograms: the input chirp
 * has unit modulus and the unnormalised DFT satisfies F^H F = nx ny I, so C of
 * Eq. (4) equals nx ny I^T I for the real interferogram matrix I, an integer Gram
 * evaluated exactly in FP64 (same entry points as HH_FP16_STORE).  Forms 1-6
 * require nt <= 32 (else HH_E_UNSUPPORTED).  Forms 1-5 also run the projection
 * of Eqs. (6)-(7) on MFMA in their operand format (unless proj_mode is
 * HH_PROJ_COMPLEMENT): the kept components as one real product per 16 pixels,
 * z = m s + r V with m the pixel's temporal mean (FP32) and only the residual r
 * rounded (a power-of-two scale per pixel for FP16 and FP8), FP32 accumulation,
 * |z|^2 summed in FP32.  The other forms project in FP32/FP64. */
enum {
  HH_FP32 = 0,      /* FP32 operands, FP32 sums of <= 512 products, FP64 reduction */
  HH_BF16 = 1,      /* BF16 operands (round to nearest even) on MFMA, FP32 accumulation */
  HH_FP16 = 2,      /* FP16 operands, one power-of-two scale per 256 pixels */
  HH_BF16X3 = 3,    /* R = hi + lo in BF16, hi*hi + hi*lo + lo*hi on MFMA */
  HH_FP16X3 = 4,    /* R = hi + lo in FP16 (scaled as HH_FP16), three MFMA products */
  HH_FP8E4M3 = 5,   /* OCP e4m3 operands, power-of-two scale per frame and 256 pixels */
  HH_FP16_STORE = 6, /* hologram stored as FP32 mean + FP16 residual (see above) */
  HH_EXACT = 7       /* covariance exactly from the frames (see hh_covariance_frames); FP32
                        hologram for the projection; nt <= 64 */
};

/* How the image of Eq. (7) is evaluated (same result up to rounding). */
enum {
  HH_PROJ_AUTO = 0,        /* the cheaper of the two below */
  HH_PROJ_DIRECT = 1,      /* sum over kept k of |sum_t H[p][t] V[t][k]|^2, FP32 */
  HH_PROJ_COMPLEMENT = 2,  /* sum_t |H[p][t]|^2 - sum over dropped k of |.|^2, FP64
                              (V unitary, Eq. (5); exact reformulation) */
  HH_PROJ_FIRST = 3        /* projection first: Y_k = Eq. (1) applied to J_k = sum_t V[t][k] I_t
                              (Eq. (1) is linear in the frame), M = sum over kept k of |Y_k|^2:
                              K transforms of combined frames, the holograms are never formed.
                              Requires precision HH_EXACT (C from the frames as well) and an
                              entry point that starts from frames (see hh_project_frames) */
};

typedef struct {
  double wavelength_m;  /* lambda > 0 (laser wavelength, set-up section) */
  double distance_m;    /* z != 0: sensor-to-object distance of Eq. (1) */
  double pitch_m;       /* d > 0: square pixel pitch (set-up section) */
  int32_t nx, ny;       /* frame width (fast axis) and height: powers of two, 8..4096 */
  int32_t nt;           /* stack length n_t, 2..64 */
  int32_t k_lo, k_hi;   /* kept components of I_f (Eq. (6)), 0-based, inclusive,
                           counted in DESCENDING eigenvalue order: 0 <= k_lo <= k_hi < nt.
                           The paper's 1-based ascending n1..n2 maps to nt-n2..nt-n1. */
  int32_t precision;    /* HH_FP32 ... HH_EXACT (covariance contraction, hologram storage) */
  int32_t proj_mode;    /* HH_PROJ_AUTO / _DIRECT / _COMPLEMENT */
  int32_t eigh_solver;  /* HH_EIGH_JACOBI (0) or HH_EIGH_TRIDIAG (1): the step (c) solver of the
                           pipeline entry points */
} hh_params;

/* Bytes of device workspace hh_pipeline needs for *p (0 if *p is invalid). */
size_t hh_workspace_bytes(const hh_params *p);

/* Bytes of device workspace hh_covariance needs for *p (0 if *p is invalid). */
size_t hh_covariance_workspace_bytes(const hh_params *p);

/* Bytes of device workspace hh_project_frames needs for *p (0 if *p is invalid). */
size_t hh_project_frames_workspace_bytes(const hh_params *p);

/*
 * Steps (d)+(e), Eq. (6)-(7), evaluated from the frames (projection first):
 * by linearity of Eq. (1) the projected hologram of component k is the Fresnel
 * transform of J_k = sum_t V[t][k] I_t, so
 *   image[p] = sum_{k = k_lo..k_hi} |Fresnel(J_k)[p]|^2,
 * the same image as hh_project_render on hh_fresnel's holograms, computed with
 * K = k_hi - k_lo + 1 transforms instead of nt and without forming H.
 *   frames : uint16 [nt][ny][nx], 16-byte aligned.
 *   evecs  : complex128 [nt][nt], evecs[t][k] = V[t][k] (any complex matrix; the
 *            eigenvectors of Eq. (5) in the intended use), 16-byte aligned.
 *   image  : float32 [ny][nx], 8-byte aligned.
 *   workspace: hh_project_frames_workspace_bytes(p) bytes, 256-byte aligned
 *            (K row-transformed components and partial images).
 * Uses the optics, nx, ny, nt, k_lo, k_hi of *p (precision and proj_mode are
 * not read).  J_k is summed in FP32 around each pixel's frame-0 value (exact
 * integer differences), the transforms and |.|^2 are FP32.  Errors as hh_pipeline.
 */
hh_status hh_project_frames(const hh_params *p, const uint16_t *frames, const double *evecs, float *image,
                            void *workspace, size_t ws_bytes, void *stream);

/*
 * Step (a), Eq. (1): Fresnel holograms of `nframes` frames.
 *   frames : uint16 [nframes][ny][nx] raw interferograms (no offset removed),
 *            16-byte aligned.
 *   holo   : complex64 [nframes][ny][nx] output,
 *            holo[t][v][u] = sum_{n,m} I_t[n][m] c[n][m] exp(-2 pi i (u m/nx + v n/ny)),
 *            c[n][m] = exp(-i pi d^2 ((m - nx/2)^2 + (n - ny/2)^2) / (lambda z)).
 *            Forward, unnormalised DFT, DC at index 0; the constant prefactor and
 *            the output-plane chirp of Eq. (1) are omitted.
 * Only wavelength, distance, pitch, nx, ny of *p are used.  nframes >= 0 (0 = no-op).
 */
hh_status hh_fresnel(const hh_params *p, const uint16_t *frames, int32_t nframes,
                     float *holo, void *stream);

/*
 * Step (b), Eq. (4): C = H^{t*} H of a hologram stack.
 *   holo : complex64 [nt][ny][nx] (e.g. the output of hh_fresnel).
 *   cov  : complex128 [nt][nt] output, C[s][t] = sum_p conj(H_s[p]) H_t[p]; exactly
 *          Hermitian (Im C[s][s] = 0, C[t][s] = conj C[s][t]); no centring, no 1/N.
 *   workspace : device buffer of at least hh_covariance_workspace_bytes(p) bytes.
 * Uses nx, ny, nt, precision of *p.
 */
hh_status hh_covariance(const hh_params *p, const float *holo, double *cov,
                        void *workspace, size_t ws_bytes, void *stream);

/*
 * hh_covariance without a workspace argument, for callers that cannot allocate
 * device memory (code under HIP graph capture, serving loops and harnesses that
 * forbid hipMalloc).  Same arguments, launch, results and errors as
 * hh_covariance; the split-K partials live in a static device array of
 * hh_covariance_noalloc_max_bytes() bytes (48 MiB), one per GPU, held until the
 * process ends.  No call allocates or frees device memory.  Sizes whose partials
 * do not fit (above about 2M pixels at nt <= 32, 0.5M at nt > 32, with the default
 * 256-pixel chunk) return HH_E_UNSUPPORTED and enqueue nothing.  Every call on a
 * GPU shares that GPU's array: calls that overlap on one GPU (other streams,
 * other threads) race and must be ordered by the caller.
 */
hh_status hh_covariance_noalloc(const hh_params *p, const float *holo, double *cov, void *stream);
size_t hh_covariance_noalloc_max_bytes(void);

/*
 * Step (b) without step (a): C of Eq. (4) computed exactly from the frames as
 * nx ny I^T I (I[p][t] the uint16 interferograms; exact because Eq. (1) as
 * discretised is a unit-modulus chirp followed by an unnormalised DFT).  Every
 * product and partial sum is an integer below 2^53, so the result is exact for
 * nx ny <= 2^21 (16-bit data) and rounded once per partial beyond; C is real
 * (imaginary parts written as 0).
 *   frames : uint16 [nt][ny][nx], 16-byte aligned.   cov : complex128 [nt][nt].
 *   workspace : at least hh_covariance_workspace_bytes(p) bytes.
 * Uses nx, ny, nt of *p (nt <= 64).
 */
hh_status hh_covariance_frames(const hh_params *p, const uint16_t *frames, double *cov,
                               void *workspace, size_t ws_bytes, void *stream);

/*
 * Step (c), Eq. (5): Hermitian eigendecomposition C = V Lambda V^{t*} in FP64
 * (parallel cyclic Jacobi, one workgroup).
 *   nt    : 2..64.
 *   cov   : complex128 [nt][nt] Hermitian input (only read).
 *   evals : float64 [nt] output, DESCENDING.
 *   evecs : complex128 [nt][nt] output, evecs[t][k] = V[t][k] (column k is the
 *           eigenvector of evals[k]); each column's phase is fixed so that its
 *           largest-modulus entry (lowest row among ties within 1e-12) is real > 0.
 *   info  : int32 [1] output on the device: number of Jacobi sweeps (>= 0), or -1
 *           if the iteration did not converge within the sweep limit (outputs
 *           are then the last iterate).
 */
hh_status hh_eigh(int32_t nt, const double *cov, double *evals, double *evecs,
                  int32_t *info, void *stream);

/* hh_eigh with an explicit sweep limit (max_sweeps >= 0; hh_eigh uses 40). */
hh_status hh_eigh_ex(int32_t nt, const double *cov, double *evals, double *evecs,
                     int32_t *info, int32_t max_sweeps, void *stream);

/*
 * Step (c) as hh_eigh, by Householder reduction of C to a real tridiagonal matrix
 * (reflectors whose phases make the off-diagonal real) followed by implicit QL
 * with shifts, in FP64, one workgroup per problem; the eigenvector phases and the
 * order are fixed as in hh_eigh.  info : number of QL iterations (>= 0), or -1 if
 * some eigenvalue needed more than max_iter (>= 0; the pipelines use 40).
 */
hh_status hh_eigh_tridiag(int32_t nt, const double *cov, double *evals, double *evecs,
                          int32_t *info, int32_t max_iter, void *stream);

/*
 * Steps (d)+(e), Eqs. (6)-(7): the power image of the kept components, with the
 * projection fused into the |.|^2 sum (the components are never stored).
 *   holo  : complex64 [nt][ny][nx].
 *   evecs : complex128 [nt][nt], evecs[t][k] = V[t][k] (as written by hh_eigh).
 *   image : float32 [ny][nx] output, M[p] = sum_{k=k_lo..k_hi} |sum_t H[p][t] V[t][k]|^2.
 * Uses nx, ny, nt, k_lo, k_hi, precision, proj_mode of *p.  HH_PROJ_COMPLEMENT
 * and HH_PROJ_AUTO rely on V being unitary (as hh_eigh returns it).  With
 * precision HH_BF16 .. HH_FP8E4M3 (nt <= 32) and proj_mode other than
 * HH_PROJ_COMPLEMENT, the kept components are projected on MFMA in that format
 * (see the precision forms above).
 */
hh_status hh_project_render(const hh_params *p, const float *holo, const double *evecs,
                            float *image, void *stream);

/*
 * The SVD-filtered stack, Eq. (3): Hf = H V I_f V^H with I_f the selector of
 * components k_lo..k_hi (descending order), i.e. the stack with the dropped
 * components removed, frame by frame, for temporal analysis downstream.  Its
 * power sum_t |Hf[p][t]|^2 is the image of Eq. (7).
 *   holo  : complex64 [nt][ny][nx], read only.
 *   evecs : complex128 [nt][nt] as written by hh_eigh (unitary).
 *   out   : complex64 [nt][ny][nx] output; must not overlap holo.  All three 16-byte aligned.
 * Uses nx, ny, nt, k_lo, k_hi, proj_mode of *p: HH_PROJ_DIRECT sums the kept
 * components in FP32; HH_PROJ_COMPLEMENT subtracts the dropped ones (coefficients
 * in FP64) from H; HH_PROJ_AUTO takes the shorter list.
 */
hh_status hh_svd_filter(const hh_params *p, const float *holo, const double *evecs, float *out,
                        void *stream);

/*
 * Steps (a)-(e) on one stack, in the paper's order, all on `stream`.
 *   frames : uint16 [nt][ny][nx], 16-byte aligned.
 *   image  : float32 [ny][nx] output (Eq. (7)).
 *   evals, evecs, info : optional outputs as in hh_eigh (NULL = not returned).
 *   workspace : at least hh_workspace_bytes(p) bytes; holds the hologram stack
 *               and the covariance partial sums.  It must not be shared by calls
 *               that may run concurrently.
 */
hh_status hh_pipeline(const hh_params *p, const uint16_t *frames, float *image,
                      double *evals, double *evecs, int32_t *info,
                      void *workspace, size_t ws_bytes, void *stream);

/* One stack of a batch: its input, its image and optional eigen-outputs. */
typedef struct {
  const uint16_t *frames; /* uint16 [nt][ny][nx], 16-byte aligned */
  float *image;           /* float32 [ny][nx] output */
  double *evals;          /* float64 [nt] output, or NULL */
  double *evecs;          /* complex128 [nt][nt] output, or NULL */
  int32_t *info;          /* int32 [1] output (solver iterations, -1 = not converged), or NULL */
} hh_stack;

/* Bytes of workspace hh_pipeline_batch needs for the n stacks described by p[0..n-1]
   (0 if any p[i] is invalid or n < 1). */
size_t hh_batch_workspace_bytes(const hh_params *p, int32_t n);

/*
 * Steps (a)-(e) on n independent stacks, possibly of different sizes and stack
 * lengths (p[i] describes stack i), all on `stream`: every stack's Fresnel
 * transform and covariance, then one launch that solves all n eigenproblems in
 * parallel (one workgroup each), then every stack's projection and image.  Each
 * stack's results are those hh_pipeline would produce for it alone.
 *   p, stacks : host arrays of n entries (read during the call only).
 *   workspace : at least hh_batch_workspace_bytes(p, n) bytes, 256-byte aligned.
 * 1 <= n <= 4096.
 */
hh_status hh_pipeline_batch(const hh_params *p, int32_t n, const hh_stack *stacks, void *workspace,
                            size_t ws_bytes, void *stream);

/* One hologram stack of hh_analyze_batch: its input, its image and optional eigen-outputs. */
typedef struct {
  const float *holo;      /* complex64 interleaved [nt][ny][nx] input (Fresnel holograms, step (a)),
                             16-byte aligned */
  float *image;           /* float32 [ny][nx] output */
  double *evals;          /* float64 [nt] output, or NULL */
  double *evecs;          /* complex128 [nt][nt] output, or NULL */
  int32_t *info;          /* int32 [1] output (solver iterations, -1 = not converged), or NULL */
} hh_window;

/* Bytes of workspace hh_analyze_batch needs for the n stacks described by p[0..n-1]
   (0 if any p[i] is invalid or n < 1). */
size_t hh_analyze_batch_workspace_bytes(const hh_params *p, int32_t n);

/*
 * Steps (b)-(e) (Eqs. (4)-(7)) on n hologram stacks the caller already holds in
 * device memory, e.g. windows of a ring of Fresnel holograms that a stream of
 * frames fills with hh_fresnel, so that frames shared by overlapping windows are
 * transformed once.  Every stack's covariance, then one launch for all n
 * eigenproblems, then every stack's projection and image; each result is what
 * hh_covariance + hh_eigh + hh_project_render give for that stack alone.
 * Uses nx, ny, nt, k_lo, k_hi, precision, proj_mode of each p[i] (the optics are
 * not read).  The holograms are only read.
 *   p, wins   : host arrays of n entries (read during the call only).
 *   workspace : at least hh_analyze_batch_workspace_bytes(p, n) bytes, 256-byte aligned.
 * 1 <= n <= 4096.  Errors as hh_pipeline_batch.
 */
hh_status hh_analyze_batch(const hh_params *p, int32_t n, const hh_window *wins, void *workspace,
                           size_t ws_bytes, void *stream);

/*
 * The work of one hh_pipeline_batch call, captured once as a HIP graph and
 * replayed with one launch (steps (a)-(e) on n uneven stacks; no allocation or
 * host work per replay).  Its schedule differs from the eager call's and not its
 * results: the stacks of the largest eigenproblem class present (n_t > 32, else
 * > 16; the first half when all are in one class) are transformed first, and their
 * eigenproblems and projections run on a second graph branch beside the transforms,
 * eigenproblems and projections of the other stacks, so the single-workgroup solves
 * overlap bandwidth-bound work.  The pointers in p/stacks/workspace are baked into the
 * graph: every replay reads the CURRENT contents of the same frame buffers and
 * rewrites the same outputs, so a caller refills the frames between replays.
 * The buffers must outlive the graph; replays on one workspace must not overlap.
 * hh_graph_create validates exactly as hh_pipeline_batch does, enqueues nothing
 * on any caller stream, and sets *out (NULL on error).
 */
typedef struct hh_graph hh_graph;
hh_status hh_graph_create(const hh_params *p, int32_t n, const hh_stack *stacks, void *workspace,
                          size_t ws_bytes, hh_graph **out);
/* One replay on `stream`; returns without synchronising. */
hh_status hh_graph_launch(hh_graph *g, void *stream);
/* Frees the graph (NULL is ignored).  Not while a replay may still run. */
void hh_graph_destroy(hh_graph *g);

/*
 * Launch choices for one problem shape.  The results do not depend on them
 * beyond rounding (every choice meets the same accuracy bar); only speed does.
 *   fft_rows : row-FFT launch shape: 0 = 16 points per thread, 256-thread groups;
 *              1 = 32 points per thread, 256-thread groups; 2 = 32 points per
 *              thread, 2 rows per group; 3 = 16 points per thread, one row per
 *              group; 4 and 5 = shapes 2 and 0 exchanging real and imaginary parts
 *              separately through half the LDS; 6 and 7 = shapes 3 and 2 as a
 *              persistent grid (as many groups as the compute units hold) that
 *              loads the next row while transforming the current one; 8 = the
 *              persistent form with 16 points per thread, 4 rows per group and the
 *              split exchange; 9 = the same with 2 rows per group and the full
 *              exchange.  Shapes 1-9 exist for nx >= 512.
 *   fft_cols : column-FFT launch shape: 0 = 16 points per thread, 16 columns per
 *              group (fewer where the LDS does not hold them); 1 = 16 points, half
 *              as many columns; 2 = 32 points per thread; 3 and 4 = shapes 0 and 2
 *              with the split exchange; 5 and 6 = shapes 0 and 3 as a persistent grid
 *              (as many groups as the compute units hold) that loads the next strip
 *              while transforming the current one; 7 = shape 4 with the twiddles
 *              staged in LDS and registers capped so that two groups share a
 *              compute unit.
 *              Shapes 1-7 exist for ny >= 512.
 *   gram_pxw : covariance split-K chunk, pixels per wavefront: 256, 512 or 1024
 *              (FP32 partial sums grow with it).
 *   gram_ref : reference m of the covariance's exact per-pixel split H = m 1^T + R
 *              (HH_FP32 form, nt <= 32): 0 = the temporal mean, 1 = the pixel's
 *              frame-0 value (one lane broadcast instead of a 16-lane sum).
 *   group    : frames per Fresnel group (row pass then column pass), 0 = about
 *              64 MiB of FP32 holograms, at most four times that (the FP16
 *              storage form clamps it to the default, the size of its buffer).
 *   fused    : HH_FP32 form of the entry points that start from frames: 1 = three
 *              passes over one hologram-sized buffer where the shape allows it
 *              (nx in {512, 1024, 2048}, ny in {512, 1024}, nt <= 32): the column
 *              transforms with one radix-4 split of the row transform, then the
 *              remaining quarter-row transforms of every frame finished in LDS and
 *              fed to the covariance, and after step (c) the same transforms fed to
 *              the projection, so H is never stored (HBM traffic: the frames once,
 *              one hologram-sized buffer written once and read twice, the image);
 *              0 (the default) = the row pass, column pass, covariance and
 *              projection on a stored H (the only form elsewhere).  The other
 *              choices above apply to the stored-H form.
 * The FFT choices, the group and fused apply to every call with the same (nx, ny)
 * on the current device, gram_pxw and gram_ref to the same (nx * ny, nt, precision).
 */
typedef struct {
  int32_t fft_rows, fft_cols, gram_pxw, group, gram_ref, fused;
} hh_tuning;

/* Choices now in force for *p (defaults where none were set).  Uses nx, ny, nt, precision. */
hh_status hh_tuning_get(const hh_params *p, hh_tuning *t);
/* Sets the choices for the shape of *p (validated; HH_E_INVALID if out of range). */
hh_status hh_tuning_set(const hh_params *p, const hh_tuning *t);
/* Forgets every choice (back to the defaults). */
void hh_tuning_reset(void);

/*
 * Autotuner: times hh_pipeline on `frames` (reps timed runs per candidate, the
 * median kept) for each launch choice in turn (row shape, column shape, group,
 * split-K chunk, each keeping the best so far), stores the fastest for the shape
 * of *p and returns it in *best (may be NULL).  Synchronous: it waits for its
 * own launches on `stream`, allocates a scratch image, and must not be called
 * under stream capture.  workspace as for hh_pipeline.  1 <= reps <= 1000.
 */
hh_status hh_autotune(const hh_params *p, const uint16_t *frames, void *workspace, size_t ws_bytes,
                      int32_t reps, hh_tuning *best, void *stream);

/*
 * Fourier demodulation, Eqs. (8)-(9) (the paper's comparison method):
 *   image[p] = sum_{f=k_lo..k_hi} |sum_t H[p][t] W[t][f]|^2,
 *   W[t][f] = exp(-2 i pi t f / nt) / sqrt(nt), 0-based frequency indices
 *   (the paper's 1-based n1..n2 maps to n1-1..n2-1).
 * holo: complex64 [nt][ny][nx] on the device (16-byte aligned); image: float32
 * [ny][nx] on the device.  A power-of-two nt <= 64 is transformed along t per
 * pixel (an FFT in registers; proj_mode is not used); any other nt is projected
 * onto the band's basis columns in the mode proj_mode.  Uses nx, ny, nt, k_lo,
 * k_hi, proj_mode of *p.
 */
hh_status hh_fourier_render(const hh_params *p, const float *holo, float *image, void *stream);

/*
 * Fourier demodulation of nwin windows of a frame stream, Eqs. (8)-(9): window w
 * takes the nt holograms holo[w*hop .. w*hop + nt - 1] and its image, images[w],
 * is the band power of hh_fourier_render (equal to it window by window).
 * holo: complex64 [(nwin - 1)*hop + nt][ny][nx] on the device (16-byte aligned);
 * images: float32 [nwin][ny][nx] on the device.  1 <= nwin <= 4096,
 * 1 <= hop <= 4096, else HH_E_INVALID (and the other checks of
 * hh_fourier_render).  One launch for every window: the frames that consecutive
 * windows share are read from the cache.
 */
hh_status hh_fourier_render_windows(const hh_params *p, const float *holo, int32_t nwin, int32_t hop, float *images,
                                    void *stream);

/* Static text for a status code. */
const char *hh_status_string(hh_status s);

/* Detail of the last failing call on the calling thread ("" if none). */
const char *hh_last_error(void);

/* Free every cached device table (call only when no work using them is in flight). */
void hh_plan_cache_clear(void);

/*
 * Kernel timing for measurement.  While enabled (on != 0), each kernel the
 * library launches is bracketed by two HIP events recorded on its own stream.
 * hh_profile_read waits for those events and writes a JSON object
 * {"kernel": [launches, total_ms], ...} into buf (NUL-terminated, truncated to
 * len); it returns the number of bytes needed.  hh_profile_reset forgets all.
 */
void hh_profile_enable(int32_t on);
int32_t hh_profile_read(char *buf, int32_t len);
void hh_profile_reset(void);

#ifdef __cplusplus
}
#endif

#endif /* HH_H */
