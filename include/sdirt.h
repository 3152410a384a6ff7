/*
 * sdirt.h -- C ABI of the MI355X (gfx950) dual-pixel PSF engine.
 *
 * The library implements the hot path of the ray-traced dual-pixel (DP)
 * simulator of "Simulating Dual-Pixel Images From Ray Tracing For Depth
 * Estimation" (He et al., ICCV 2025):
 *   - Sec. 3.1: a ray set from an object point toward samples of the
 *     entrance pupil, refracted through every lens surface by Snell's law
 *     to the sensor; each landed ray split into the left or right
 *     sub-pixel (microlens model, Eq. (1)/(2) with Eq. (S1) parameters, or
 *     a smooth angular response) and accumulated into PSF_L / PSF_R,
 *     Eq. (3);
 *   - Sec. 3.2 and Supplement S1.3: the pixel-wise local convolution that
 *     renders the left/right images from an all-in-focus image with each
 *     pixel's own DP PSF;
 *   - hand-written adjoints of both, and the PSF surrogate MLP of Sec. 3.2
 *     and Supplement S1.4 with bf16 matrix-core kernels.
 *
 * Conventions shared by every entry point
 *   - Lengths in millimetres, wavelengths in micrometres, z = 0 at the
 *     first vertex, light toward +z, object depths measured from the first
 *     vertex toward -z.
 *   - Host structs (and the host arrays they point to) are read only during
 *     the call.  Arrays documented as "device" are caller-owned device
 *     buffers; the library keeps no pointer after returning.
 *   - `stream` is a hipStream_t (NULL = the default stream).  Every call is
 *     asynchronous on that stream: it validates, precomputes on the host,
 *     enqueues kernels and returns; it never synchronises.  The library has
 *     no global mutable device state, so calls on different streams may
 *     overlap.  Output buffers are cleared by the library's own kernels.
 *   - Return value: SDIRT_OK (0) or a negative status.  Per-ray optical
 *     failures (miss, clipping, total internal reflection, asphere root
 *     failure, invalid direction) are not errors: they are counted in the
 *     per-point statistics.
 */
#ifndef SDIRT_H
#define SDIRT_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

/* ---- status codes ---------------------------------------------------- */
#define SDIRT_OK              0
#define SDIRT_EINVAL         -1   /* bad argument: NULL, size, range, NaN  */
#define SDIRT_EUNSUPPORTED   -2   /* valid but unsupported mode/dtype/size */
#define SDIRT_ELAUNCH        -3   /* a HIP launch or runtime call failed   */
#define SDIRT_ENODEVICE      -4   /* no HIP device available               */
#define SDIRT_ESCRATCH       -5   /* needs more than the static scratch    */

/* ---- limits ----------------------------------------------------------- */
#define SDIRT_MAX_SURFACES    24  /* rows of the prescription incl. stop   */
#define SDIRT_MAX_LAMBDAS      4  /* distinct wavelengths per call         */
#define SDIRT_MAX_FIELDS      64  /* grid-mode fields                      */
#define SDIRT_MAX_DEPTHS      64  /* grid-mode depths                      */
#define SDIRT_MAX_KS         129  /* PSF window (odd)                      */
#define SDIRT_MAX_BANK_F      64
#define SDIRT_MAX_BANK_D      64

/* ---- lens prescription (Table S1 / S2 columns) ------------------------ */
enum { SDIRT_SPHERE = 0, SDIRT_PLANE = 1, SDIRT_STOP = 2, SDIRT_ASPHERE = 3,
       SDIRT_IDEAL = 4 };
enum { SDIRT_MAT_CAUCHY = 0,   /* n = p0 + p1 / lambda^2                  */
       SDIRT_MAT_ABBE = 1 };   /* p0 = n_d, p1 = V_d (d/F/C-line Cauchy)  */

typedef struct {
    int    kind;           /* SDIRT_SPHERE ... SDIRT_IDEAL                  */
    int    material;       /* model of the medium AFTER this surface        */
    double mat_p0, mat_p1; /* its parameters (air: CAUCHY 1, 0)             */
    double c;              /* curvature 1/R (1/mm); ignored for PLANE/STOP  */
    double t;              /* axial distance to the next vertex (mm); for
                              the last surface: sensor distance, used unless
                              focus_depth > 0                               */
    double semi_diameter;  /* clear semi-diameter (mm); the stop's radius   */
    double conic;          /* k (ASPHERE)                                   */
    double asph[5];        /* a4, a6, a8, a10, a12 (ASPHERE)                */
    double focal;          /* IDEAL only: focal length (mm)                 */
} sdirt_surface;

typedef struct {
    int n_surfaces;                  /* 1 .. SDIRT_MAX_SURFACES             */
    int stop;                        /* index of the aperture stop          */
    const sdirt_surface* surfaces;   /* host array [n_surfaces]             */
    int    object_material;          /* medium before surface 0             */
    double object_p0, object_p1;
    double f_number;        /* > 0: stop resized so that the paraxial
                               entrance pupil diameter is EFL / f_number   */
    double focus_depth;     /* > 0: sensor at the paraxial image of the
                               on-axis point at this depth                 */
    double ref_wavelength;  /* wavelength of the stop / focus / chief-ray
                               magnification computation (um, > 0)         */
} sdirt_lens;

/* First-order data resolved by the host (paraxial, at ref_wavelength). */
typedef struct {
    double efl;             /* effective focal length                      */
    double bfd;             /* back focal distance (infinity focus)         */
    double sensor_distance; /* last vertex -> sensor plane                  */
    double stop_radius;     /* possibly resized by f_number                 */
    double z_ep, rho_ep;    /* entrance pupil position / radius             */
    double m_num;           /* chief-ray magnification m(d) = m_num/(z_ep+d) */
    double sensor_z;        /* sensor plane z (from vertex 0)               */
} sdirt_lens_info;

/* ---- dual-pixel sensor (Sec. 3.1, Eq. (S1)) --------------------------- */
enum { SDIRT_DP_SIGMOID = 0, SDIRT_DP_MICROLENS = 1 };

typedef struct {
    double pitch;          /* DP pixel size ps (mm)                         */
    int    dp_mode;
    double sigmoid_k;      /* left weight = logistic(k * sin(theta_x))     */
    double ml_h, ml_f, ml_w, ml_r;  /* microlens model, units of pitch;
                                       requires 0 <= h < f, w > 0, r > 0   */
} sdirt_sensor;

/* ---- PSF query -------------------------------------------------------- */
enum { SDIRT_SPLAT_BOX = 0, SDIRT_SPLAT_TENT = 1 };
enum { SDIRT_NORM_NONE = 0, SDIRT_NORM_SUM = 1, SDIRT_NORM_MAX = 2 };
enum { SDIRT_F32 = 0, SDIRT_F64 = 1, SDIRT_BF16 = 2 };

typedef struct {
    /* Grid mode: P = F * D * L points, index q = (f * D + d) * L + l.      */
    int n_fields, n_depths, n_wavelengths;
    const double* fields;       /* host [F][2] image-plane (h_x, h_y), mm   */
    const double* depths;       /* host [D] object depths (mm, > 0)         */
    const double* wavelengths;  /* host [L] (um, > 0); also the slots of
                                   list mode                               */
    /* List mode (used when points != NULL): P = n_points arbitrary points. */
    int n_points;
    const double* points;       /* device [P][4]: h_x, h_y, depth, slot
                                   (slot = index into wavelengths)          */
    int rays_x, rays_y;         /* stratified pupil grid, rays = x * y      */
    uint32_t seed;
    int jitter;                 /* 0: cell centres                         */
    int ks;                     /* odd window size                         */
    int splat;                  /* SDIRT_SPLAT_*                           */
    int normalize;              /* SDIRT_NORM_*                            */
    int out_dtype;              /* SDIRT_F32 or SDIRT_F64                  */
    int math;                   /* SDIRT_F64 (default) or SDIRT_F32 trace  */
    int deterministic;          /* 1: bitwise reproducible PSFs (below)    */
} sdirt_psf_query;

/* Resolve stop size, sensor position and pupil on the host (no device
 * work; usable without a GPU).  See Sec. 3.1 (entrance pupil) and Sec. 5.1
 * (F-number, focus distance). */
int sdirt_resolve_lens(const sdirt_lens* lens, sdirt_lens_info* out);

/* Entrance pupil (z, radius) at a given wavelength with the resolved stop;
 * host only. */
int sdirt_pupil(const sdirt_lens* lens, double wavelength, double* z_ep,
                double* rho_ep);

/* Trace given rays surface by surface (Sec. 3.1; parity and debugging).
 *   o, d      device [n][3] doubles: origin (global frame) and unit direction
 *   hits_out  device [n][S+1][6] doubles: per surface the vertex-local hit
 *             point (x, y, z) and the direction after the surface; entry S
 *             is the sensor plane (x, y, 0, direction).
 *   status    device [n] int: 0 alive, 1 miss, 2 clip, 3 TIR, 4 asphere
 *             root failure, 5 invalid; first failure wins.
 * math selects the arithmetic of the trace (SDIRT_F64 or SDIRT_F32). */
int sdirt_trace_rays(const sdirt_lens* lens, double wavelength, int math,
                     int n, const double* o, const double* d,
                     double* hits_out, int* status_out, void* stream);

/* DP PSFs of a query, Eq. (3) (Sec. 3.1), with the pupil sampling,
 * trace, DP split, splat and normalisation of the hot path.
 *   psf_out    device [P][2][ks][ks], f32 or f64 (query->out_dtype); side 0
 *              = left, row i toward +y, column j toward +x, centred on the
 *              field point.
 *   stats_out  device [P][7] doubles (may be NULL): launched, vignetted,
 *              transmitted, left-in-window, right-in-window,
 *              missed-sub-pixel, outside-window energies (before
 *              normalisation).
 * Both buffers are overwritten.  By default the rays of a point are split
 * over several workgroups whose float32 tiles are added with atomics, so
 * PSF values vary from run to run in the last bits (~1e-7 relative).  With
 * query->deterministic = 1 each ray's weight is rounded to a multiple of
 * 2^-32 and summed in 64-bit integers (order-free, exact), and each point
 * is traced by a single workgroup, so repeated calls give identical bits;
 * the integer tile needs 16 ks^2 bytes of LDS, so ks <= 101 in that mode
 * (SDIRT_EUNSUPPORTED above), and the chunk count of
 * sdirt_trace_dp_psf_chunks is ignored. */
int sdirt_trace_dp_psf(const sdirt_lens* lens, const sdirt_sensor* sensor,
                       const sdirt_psf_query* query, void* psf_out,
                       double* stats_out, void* stream);

/* sdirt_trace_dp_psf with the number of ray chunks per point given by the
 * caller instead of chosen by the library (Sec. 3.1; the result is the same
 * estimator, Eq. (3), for any chunk count).  A point's pupil grid is cut
 * into `chunks` contiguous ranges of ray indices, each traced by one
 * workgroup whose LDS tile is added into psf_out with float32 atomics; the
 * launch has chunks * P workgroups.  chunks >= 1 (SDIRT_EINVAL otherwise);
 * values above the ray count are clamped to it; ignored in deterministic
 * mode (one workgroup per point).  Other arguments, layouts, ownership and
 * errors as sdirt_trace_dp_psf.  For sweeping launch shapes and for tests
 * that the chunking does not change the PSFs. */
int sdirt_trace_dp_psf_chunks(const sdirt_lens* lens, const sdirt_sensor* sensor,
                              const sdirt_psf_query* query, void* psf_out,
                              double* stats_out, int chunks, void* stream);

/* Number of parameters of the trace adjoint: 8 * n_surfaces + 1. */
int sdirt_n_params(const sdirt_lens* lens);

/* Adjoint of sdirt_trace_dp_psf (TENT splat, SIGMOID response, NORM_NONE,
 * grid mode) under frozen framing: pupil samples, pupil, window centres and
 * the set of surviving rays are those of the given parameters.
 *   grad_psf        device [P][2][ks][ks] f32: dL/dPSF
 *   grad_params_out device [8 S + 1] doubles, overwritten: per surface
 *                   [c, t, conic, a4, a6, a8, a10, a12] (t of the last
 *                   surface = sensor distance), then the response slope k.
 * Each ray is re-traced forward in registers and swept in reverse; per-ray
 * derivatives are reduced in the wave before global atomics. */
int sdirt_trace_dp_psf_backward(const sdirt_lens* lens,
                                const sdirt_sensor* sensor,
                                const sdirt_psf_query* query,
                                const float* grad_psf,
                                double* grad_params_out, void* stream);

/* ---- pixel-wise DP renderer (Sec. 3.2, Supplement S1.3) ---------------
 * out[n, s*C + c, y, x] = sum_{i,j} K[n,y,x,c',s][i][j] *
 *                         img[n, c, clamp(y+pad-i), clamp(x+pad-j)]
 * pad = (ks-1)/2, s = 0 left / 1 right, c' = c (per-channel kernels) or 0
 * (shared kernel).  Sources of K:
 *   DENSE: psf device [N][H][W][Cp][2][ks][ks] (f32 or bf16);
 *   BANK : psf device [F][D][L][2][ks][ks] f32 traced on radial fields
 *          along +x; per pixel the nearest field radius and nearest
 *          inverse depth of depth[n][y][x] are taken, channel c uses
 *          wavelength slot lambda_of_channel[c]; pixels left of the centre
 *          use the column-flipped kernel with sides swapped, pixels below
 *          it the row-flipped kernel (an approximation off the x axis).
 *   BANK2D: psf device [Fy][Fx][D][L][2][ks][ks] f32 traced on a 2-D grid
 *          of the first quadrant (h_x = field_radii[fx] >= 0, h_y =
 *          field_y[fy] >= 0) and reused in the others through the flip
 *          symmetries of DP PSFs about both axes (Sec. 5.1): per pixel the
 *          nearest grid point to (|h_x|, |h_y|), the same column flip with
 *          side swap for h_x < 0 and row flip for h_y < 0, and linear
 *          interpolation in inverse depth, in float32: iv = 1 / depth,
 *          d0 = the last plane k <= D-2 with (float)inv_depths[k] <= iv (0
 *          if none), w = clamp((iv - iv_d0) / (iv_d0+1 - iv_d0), 0, 1) (0 when
 *          D = 1); K = (1 - w) K[d0] + w K[d0 + 1].  h_x of pixel x is
 *          (x - (W-1)/2) * pitch (h_y likewise); nearest-point decisions are
 *          made exactly on the integer |2x - (W-1)| against
 *          floor(2 * midpoint / pitch).  Only window sizes 21, 31, 33, 41, 63
 *          and 65 (SDIRT_EUNSUPPORTED otherwise). */
enum { SDIRT_SRC_DENSE = 0, SDIRT_SRC_BANK = 1, SDIRT_SRC_BANK2D = 2 };

typedef struct {
    int N, C, H, W, ks;
    int source;               /* SDIRT_SRC_*                               */
    int psf_channels;         /* DENSE: Cp = 1 or C                        */
    int psf_dtype;            /* DENSE: SDIRT_F32 or SDIRT_BF16; banks: F32 */
    int bank_fields, bank_depths, bank_lambdas;
    const double* field_radii;   /* host [F], strictly increasing (mm); the
                                    x grid (Fx = bank_fields) for BANK2D    */
    const double* inv_depths;    /* host [D], strictly increasing (1/mm)   */
    int lambda_of_channel[4];    /* banks: slot per image channel          */
    double pitch;                /* banks: pixel pitch (mm)                */
    int bank_fields_y;           /* BANK2D: Fy                             */
    const double* field_y;       /* BANK2D: host [Fy], strictly increasing */
    int bank_math;               /* banks: SDIRT_BANK_FP32 (default) or
                                    SDIRT_BANK_SPLIT_BF16                   */
} sdirt_render_desc;

/* Arithmetic of the bank render and its image adjoint (SDIRT_SRC_BANK /
 * BANK2D at the matrix-core window sizes ks = 21, 31, 33, 41, 63, 65;
 * Supplement S1.3's per-pixel convolution): SDIRT_BANK_FP32 multiplies
 * float32 kernels and image values (or output gradients) on the fp32 matrix
 * cores; SDIRT_BANK_SPLIT_BF16 splits each into bf16 hi + lo parts and sums
 * the three products hi*hi + hi*lo + lo*hi on the bf16 matrix cores with
 * float32 accumulation (a product's error is below 3 * 2^-18 of its
 * magnitude; a sum's error is bounded by that fraction of the sum of the
 * products' magnitudes).  The gradient with respect to the bank, and every
 * other window size, use float32 arithmetic in either case. */
enum { SDIRT_BANK_FP32 = 0, SDIRT_BANK_SPLIT_BF16 = 1 };

/* img device [N][C][H][W] f32; depth device [N][H][W] f32 (BANK only, may
 * be NULL for DENSE); out device [N][2C][H][W] f32, overwritten.  The
 * dense source, and the radial bank at window sizes other than those of
 * the matrix-core path, stage C (ks + 7)^2 image floats per 8 x 8 pixel
 * tile in LDS: SDIRT_EUNSUPPORTED when that exceeds 160 KB (ks > 109 at
 * C = 3; every ks <= SDIRT_MAX_KS fits at C = 1).  All render calls
 * return SDIRT_EUNSUPPORTED when 8 N ceil(H / 8) ceil(W / 8) exceeds
 * 2^32 - 1 (the launch grid of the dense kernels). */
int sdirt_render_dp(const sdirt_render_desc* desc, const float* img,
                    const void* psf, const float* depth, float* out,
                    void* stream);

/* Adjoint with respect to the image: grad_img = R^T grad_out, clamped taps
 * folding onto the border pixels.  grad_out device [N][2C][H][W] f32;
 * grad_img device [N][C][H][W] f32, overwritten. */
int sdirt_render_dp_backward(const sdirt_render_desc* desc, const void* psf,
                             const float* depth, const float* grad_out,
                             float* grad_img, void* stream);

/* Gradient with respect to the kernels (the renderer of Sec. 3.2 / S1.3 is
 * linear in them).  Dense source: for every pixel, kernel channel c' and
 * side s,
 *   grad_psf[n, y, x, c', s, i, j] = sum over the image channels c that
 *       read kernel c' of grad_out[n, s*C + c, y, x]
 *                          * img[n, c, clamp(y+pad-i), clamp(x+pad-j)],
 * device [N][H][W][Cp][2][ks][ks] in desc->psf_dtype (bf16 rounded to
 * nearest even); depth is not read (may be NULL); the same LDS limit as the
 * dense forward (C (ks + 7)^2 floats <= 160 KB).  Bank sources: the sum of
 * those per-pixel gradients over the pixels that read each bank entry, the
 * lookup's mirrors undone and (BANK2D) weighted by the depth blend, device
 * f32 in the bank's own layout; depth required; window sizes 21, 31, 33,
 * 41, 63 and 65 only.  Chains the render to whatever produced the kernels
 * (the surrogate network, the tracer's adjoint).  grad_psf is overwritten. */
int sdirt_render_dp_psf_backward(const sdirt_render_desc* desc, const float* img,
                                 const float* depth, const float* grad_out,
                                 void* grad_psf, void* stream);

/* ---- PSF surrogate MLP (Sec. 3.2, Supplement S1.4) ---------------------
 * Maps an image-plane point, inverse depth and wavelength to the jointly
 * sum-normalised left/right PSF: Fourier encoding (sin / cos of
 * 2^k pi v, k < n_freq, for the four inputs mapped to [-1, 1]), n_hidden
 * ReLU layers of `width`, a linear layer to n_out = 2 ks ks logits and a
 * softmax over all of them.  Training minimises, averaged over the batch,
 * either (loss = SDIRT_LOSS_L2MAX) the L2 loss of Eq. (4) with each
 * sample's squared error scaled by the largest value of its target PSF
 * (max-normalised targets), or (SDIRT_LOSS_KL) the Kullback-Leibler
 * divergence sum_i t_i log(t_i / p_i) of the prediction from the target
 * distribution, whose logit gradient (p - t) does not vanish where the
 * network predicts no energy.
 * Parameters: one float32 vector, per layer W [out][in] row-major then
 * b [out], layers in order (sizes from sdirt_mlp_n_params).  Matrix
 * products run in bf16 on the matrix cores with float32 accumulation.
 * workspace: caller-owned device memory of sdirt_mlp_workspace_size(batch)
 * bytes for batches of `batch` rows (a multiple of 64); it holds the bf16
 * weights, activations and gradients of one batch. */
enum { SDIRT_LOSS_L2MAX = 0, SDIRT_LOSS_KL = 1 };

typedef struct {
    int n_hidden;            /* ReLU layers                                */
    int width;               /* hidden width, multiple of 64               */
    int n_out;               /* outputs, 2 * ks * ks                       */
    int n_freq;              /* frequencies per input (features 8 n_freq)  */
    double x_half, y_half;   /* h_x, h_y scale: image half-size (mm)       */
    double iv_lo, iv_hi;     /* inverse-depth range (1/mm)                 */
    double lam_lo, lam_hi;   /* wavelength range (um)                      */
    int loss;                /* SDIRT_LOSS_L2MAX or SDIRT_LOSS_KL          */
} sdirt_mlp_desc;

int sdirt_mlp_n_params(const sdirt_mlp_desc* desc, long long* n_params);
int sdirt_mlp_workspace_size(const sdirt_mlp_desc* desc, int batch, size_t* bytes);

/* Inference of n_rows inputs x (device [n_rows][4]: h_x, h_y, 1/d, lambda)
 * into out (device [n_rows][n_out], SDIRT_F32 or SDIRT_BF16) with a
 * workspace sized for ws_batch rows.  Width-256 networks run fused, in
 * chunks of as many rows as the workspace's activation area holds (512 B
 * per row; a workspace for 65536 rows holds over 10^6); other widths in
 * chunks of ws_batch rows. */
int sdirt_mlp_forward(const sdirt_mlp_desc* desc, const float* params,
                      long long n_rows, const float* x, void* out, int out_dtype,
                      void* workspace, int ws_batch, void* stream);

/* Allocation-free sdirt_mlp_forward, for callers that cannot allocate
 * device memory (code under stream capture, tight serving loops, harnesses
 * that forbid hipMalloc).  Same result as sdirt_mlp_forward (the same
 * kernels; rows are independent, so the chunking does not change any
 * value), but its working memory (the bf16 weights in fragment order and one
 * chunk of hidden activations) is a static device array of
 * SDIRT_NOALLOC_SCRATCH_BYTES inside the library instead of a caller
 * workspace; the call allocates nothing.  Each device the library runs on
 * holds its own copy of that array until the process ends.  All calls on one
 * device share it: calls that overlap on one device (other streams or host
 * threads) race and must be serialised by the caller.  Only width-256
 * networks (the fused kernels), SDIRT_EUNSUPPORTED otherwise; a network
 * whose bf16 weights plus 64 rows of activations exceed the array returns
 * SDIRT_ESCRATCH (the 5 x 256 network with 2 x 33 x 33 outputs needs
 * 1.8 MB; rows are processed in chunks of up to 65536).
 *   x device [n_rows][4] f32, out device [n_rows][n_out] f32 or bf16
 *   (out_dtype), params device f32 as for sdirt_mlp_forward. */
#define SDIRT_NOALLOC_SCRATCH_BYTES (16u << 20)
int sdirt_mlp_forward_noalloc(const sdirt_mlp_desc* desc, const float* params,
                              long long n_rows, const float* x, void* out, int out_dtype,
                              void* stream);

/* DP PSFs of a list-mode query from the surrogate network, with the ray
 * tracer as its fallback (Sec. 3.2, Supplement S1.4: the network is trained
 * on traced PSFs, and the tracer remains the reference that judges its
 * error).  The caller gives the network's measured error per band of
 * inverse depth (e.g. its held-out energy L1 against many-ray traces):
 * band_edges host [n_bands + 1] strictly increasing inverse depths (1/mm),
 * band_error host [n_bands].  Every point whose 1/depth lies in a band with
 * band_error <= max_error takes the network's PSF (softmax output, float32,
 * as sdirt_mlp_forward); every other point (in a band above the bar, or
 * outside [band_edges[0], band_edges[n_bands]]) is ray traced as by
 * sdirt_trace_dp_psf.  Band b of a point is the one with
 * band_edges[b] <= 1/depth < band_edges[b + 1] (the last band includes its
 * upper edge), 1/depth computed in float64.
 *   query     list mode (points != NULL, device [P][4]: h_x, h_y, depth,
 *             slot), normalize = SDIRT_NORM_SUM, out_dtype = SDIRT_F32
 *             (SDIRT_EUNSUPPORTED otherwise), 2 ks^2 = desc->n_out; the
 *             network input of a point is (h_x, h_y, 1/depth,
 *             wavelengths[slot]) in float32;
 *   psf_out   device [P][2][ks][ks] f32, overwritten;
 *   source_out device [P] int32, overwritten: 0 network, 1 traced;
 *   workspace as for sdirt_mlp_forward with ws_batch rows.
 * The network must have width 256.  SDIRT_EINVAL for NULL buffers, bands
 * that are not increasing or finite, n_bands outside [1, 64], a negative or
 * non-finite max_error. */
int sdirt_psf_hybrid(const sdirt_mlp_desc* desc, const float* params,
                     const sdirt_lens* lens, const sdirt_sensor* sensor,
                     const sdirt_psf_query* query, int n_bands,
                     const double* band_edges, const double* band_error,
                     double max_error, float* psf_out, int* source_out,
                     void* workspace, int ws_batch, void* stream);

/* The surrogate render (Fig. 2(c); Sec. 3.2): every pixel of an image
 * rendered with the PSF the network predicts for it, without the dense PSF
 * map ever reaching memory.  For each image n, channel c and pixel (y, x)
 * the network's softmax output P for the input (h_x, h_y, 1/d, lambda_c),
 * read as [2][ks][ks], gives
 *   out[n, s*C + c, y, x] = sum_{i,j} P[s][i][j]
 *                           * img[n, c, clamp(y+pad-i), clamp(x+pad-j)],
 * i.e. sdirt_mlp_forward into a float32 dense map followed by
 * sdirt_render_dp with per-channel kernels, with the inputs formed in
 * float32 as h_x = (x - (W-1)/2) * pitch, h_y = (y - (H-1)/2) * pitch,
 * 1/d = 1.0f / depth[n, y, x] (depth in mm), lambda_c = wavelength[c] (um).
 * The network must have width 256 and n_out = 2 ks ks (odd ks <= 65).
 * img device [N][C][H][W] f32, depth device [N][H][W] f32, out device
 * [N][2C][H][W] f32 (overwritten); workspace as for sdirt_mlp_forward with
 * ws_batch rows (a multiple of 64).  Rows are pixels, 64 per 8 x 8 tile of
 * one channel, processed in chunks of as many rows as the workspace's
 * activation area holds (512 B per row). */
typedef struct {
    int N, C, H, W;          /* images, channels (1..4), rows, columns      */
    int ks;                  /* PSF window (n_out = 2 ks ks)                 */
    double pitch;            /* pixel pitch (mm)                              */
    double wavelength[4];    /* wavelength of each channel (um)               */
} sdirt_mlp_render_desc;

int sdirt_mlp_render(const sdirt_mlp_desc* desc, const float* params,
                     const sdirt_mlp_render_desc* render, const float* img,
                     const float* depth, float* out, void* workspace, int ws_batch,
                     void* stream);

/* Loss and its gradient for one batch: grads_out device [n_params] f32,
 * loss_out device [1] f32 (either may be NULL); target device
 * [batch][n_out], each row a jointly sum-normalised PSF. */
int sdirt_mlp_backward(const sdirt_mlp_desc* desc, const float* params, int batch,
                       const float* x, const float* target, float* grads_out,
                       float* loss_out, void* workspace, void* stream);

/* Vector-Jacobian product of the network (Sec. 3.2): for n_rows inputs x
 * (device [n_rows][4], as for sdirt_mlp_forward) and an upstream gradient
 * grad_psf = dL/dP of a scalar L with respect to the softmax outputs
 * (device [n_rows][n_out] f32, e.g. the kernel-map gradient of
 * sdirt_render_dp_psf_backward for a map the network predicted), the
 * gradient of L with respect to the parameters, summed over the rows:
 * through the softmax, dL/dz_i = P_i (g_i - sum_j P_j g_j); then as
 * sdirt_mlp_backward.  grads_out device [n_params] f32 and value_out
 * device [1] f32 (sum over rows of <g, P>; may be NULL) are overwritten.
 * Rows are processed in chunks of ws_batch (a multiple of 64) with a
 * workspace sized for ws_batch; a ragged last chunk is padded in the
 * workspace with rows that contribute nothing.  n_rows = 0 gives zeros. */
int sdirt_mlp_vjp(const sdirt_mlp_desc* desc, const float* params, long long n_rows,
                  const float* x, const float* grad_psf, float* grads_out, float* value_out,
                  void* workspace, int ws_batch, void* stream);

/* One Adam update (beta1 0.9, beta2 0.999, eps 1e-8; step counts from 1) of
 * params with moments m, v (device [n_params] f32 each, updated). */
int sdirt_mlp_adam(const sdirt_mlp_desc* desc, float* params, float* m, float* v,
                   const float* grads, int step, float lr, void* stream);

/* One training step on a caller-given batch (Sec. 3.2, Eq. (4); Supplement
 * S1.4): forward, the loss of desc->loss and its gradient (as
 * sdirt_mlp_backward), then one Adam update of params with moments m, v (as
 * sdirt_mlp_adam, bias correction of step `step` >= 1, learning rate lr).
 *   x       device [batch][4] inputs, target device [batch][n_out] jointly
 *           sum-normalised PSFs (batch a multiple of 64);
 *   params, m, v  device [n_params] f32, updated in place;
 *   loss_out device [1] f32, the batch loss before the update (may be NULL);
 *   workspace as for sdirt_mlp_backward (sdirt_mlp_workspace_size(batch)).
 * SDIRT_EINVAL for NULL buffers, a batch that is not a positive multiple of
 * 64, step < 1 or a non-finite lr. */
int sdirt_mlp_train_step(const sdirt_mlp_desc* desc, float* params, float* m, float* v,
                         int step, float lr, int batch, const float* x, const float* target,
                         float* loss_out, void* workspace, void* stream);

/* n_steps training steps on a device-resident dataset (x_all [n][4],
 * t_all [n][n_out]): each step draws `batch` samples by a counter hash of
 * (seed, step, row), runs forward, loss gradient and Adam with the learning
 * rate lr_min + (lr0 - lr_min) (1 + cos(pi step / total_steps)) / 2.
 * loss_trace device [n_steps] f32 or NULL receives each step's loss. */
int sdirt_mlp_train(const sdirt_mlp_desc* desc, float* params, float* m, float* v,
                    int step0, int n_steps, float lr0, float lr_min, int total_steps,
                    int batch, long long n_samples, const float* x_all,
                    const float* t_all, uint32_t seed, float* loss_trace,
                    void* workspace, void* stream);

/* ---- measurement ------------------------------------------------------
 * Not part of the method: a kernel of known float64 FMA count, for
 * calibrating the profiler's float64 FLOP and VALU counters against the
 * trace, whose FLOPs are counted from its algorithm.  n_threads threads
 * (workgroups of 256) each run 8 independent chains of `iters` dependent
 * fused multiply-adds: exactly 8 * iters * n_threads v_fma_f64
 * (16 * iters * n_threads FLOPs).  out device [n_threads] doubles
 * (overwritten, one value per thread).  SDIRT_EINVAL for NULL out,
 * n_threads < 1 or iters < 1. */
int sdirt_calib_fma64(long long n_threads, int iters, double* out, void* stream);

/* ---- misc ------------------------------------------------------------- */
const char* sdirt_status_string(int status);
int sdirt_version(void);

#ifdef __cplusplus
}
#endif
#endif /* SDIRT_H */
