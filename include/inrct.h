/*
 * inrct.h -- C ABI of the memory-efficient INR gradient step for CT
 * (Najaf & Ongie, "Memory-efficient optimization of implicit neural
 * representations for CT reconstruction").
 *
 * The library evaluates the problem of Eq. (1), min_theta L(P{f_theta}, y),
 * with the gradient of Algorithm 1 (Eq. (2) and Eq. (3)):
 *   u = E{f_theta}      grid evaluation of the INR on the FOV  (inr_eval_grid)
 *   z = P u             ray-driven Joseph projector             (ct_project)
 *   r = dL/dz           LS residual z - y (FLS: ramp-filtered)  (inrct_residual_loss)
 *   v = P^T r           matched voxel-driven adjoint            (ct_backproject)
 *   I                   uniform k-subset of the FOV points      (inrct_sample)
 *   g = (n/k) sum_{i in I} v_i grad f_theta(x_i)                (inr_vjp_subsampled)
 *   theta <- Adam(theta, g)                                     (inrct_adam)
 * and all of it in one call on a context (inr_grad_step).
 *
 * Conventions for every entry point
 *  - Pointers named as device pointers must point to device memory of the
 *    current HIP device; the caller owns them.  Host pointers are read
 *    before the call returns and may be freed afterwards.
 *  - Calls that take a hipStream_t only enqueue work on that stream; none
 *    synchronises with the host or the device and none allocates device
 *    memory.
 *  - Device memory: every handle (geometry, model, context) keeps its
 *    tables and scratch in one workspace of exactly
 *    inrct_workspace_bytes(...) bytes, which the caller passes to the
 *    *_create call (`ws`, `ws_bytes`: device memory, 256-byte aligned, owned
 *    by the caller and kept alive until the handle is destroyed).  With
 *    ws == NULL the create call allocates that workspace itself and the
 *    destroy call frees it; nothing else in the library allocates.  A create
 *    call enqueues its table uploads and fills on its `stream`; work that
 *    uses the handle must be ordered after that stream.
 *  - Outputs are overwritten, never accumulated into.
 *  - A handle's scratch may be used by one stream at a time.  Calls that
 *    overlap on different streams must use different handles.
 *  - Every entry point returns INRCT_OK (0) or a negative status; after an
 *    error, inrct_last_error() returns a message (thread-local).  Argument
 *    errors are detected on the host before anything is enqueued.
 *  - Results are deterministic: no kernel uses atomics; every reduction has
 *    a fixed order.
 *
 * Data layouts (all float32 unless stated)
 *  - grid arrays (u, v): [N][N] (2D) or [N][N][N] (3D), x fastest; the grid
 *    spans [-1, 1]^d with pitch h = 2/N and centres -1 + (i + 1/2) h.
 *  - FOV: the disc x^2 + y^2 <= 1 (2D) or that disc at every z (3D); the n
 *    FOV points are ranked by ascending grid index.
 *  - projection arrays (y, z, r): [V][Nu] (2D) or [V][Nv][Nu] (3D), u fastest.
 *  - INR parameters theta: for each affine layer in order, W (fan_out x
 *    fan_in, row-major) then b, output layer last.  FFN layer 1 reads the
 *    encoding [sin(2 pi B x); cos(2 pi B x)] (sin block first); B is
 *    float32 [F][d], not trained.  HASH: the encoding's tables [Lh][T][2]
 *    come first (they are trained), then the MLP.
 *  - index sets: int32 grid linear indices, distinct, inside the FOV,
 *    ascending.
 */
#ifndef INRCT_H
#define INRCT_H

#include <stddef.h>
#include <stdint.h>
#include <hip/hip_runtime_api.h>

#ifdef __cplusplus
extern "C" {
#endif

/* status codes */
#define INRCT_OK 0
#define INRCT_EINVAL (-1)   /* bad argument, shape or handle               */
#define INRCT_ENOTSUP (-2)  /* unsupported geometry / architecture / dtype */
#define INRCT_EHIP (-3)     /* HIP runtime error (message has the detail)  */
#define INRCT_ENOMEM (-4)   /* device allocation failed in a *_create      */

/* geometry kinds */
#define INRCT_PAR2D 1       /* 2D parallel beam                            */
#define INRCT_CONE3D 2      /* 3D circular cone beam, flat detector        */
#define INRCT_FAN2D 3       /* 2D fan beam, flat detector (Sec. IV-A)      */

/* INR kinds and MLP precision */
#define INRCT_FFN 1         /* Fourier features + ReLU MLP                 */
#define INRCT_SIREN 2       /* sine-activated MLP                          */
#define INRCT_HASH 3        /* multi-resolution hash encoding + ReLU MLP   */
#define INRCT_FP32 0        /* FP32 matrix cores                           */
#define INRCT_BF16 1        /* BF16 matrix cores, FP32 accumulation        */

/* losses (Sec. II) */
#define INRCT_LS 0          /* 1/2 ||z - y||^2                             */
#define INRCT_FLS 1         /* 1/2 (z - y)^T F (z - y), F = ramp filter    */

/* how inr_grad_step forms v (both give the same g) */
#define INRCT_V_FULL 0      /* v = P^T r on the whole grid, then gather v_I */
#define INRCT_V_AT_I 1      /* evaluate (P^T r)_i only for i in I           */

typedef struct {
    int dim;                /* 2 or 3                                       */
    int n;                  /* points per axis N (1..4096)                  */
} inr_grid;

/* Scan geometry.  View j sits at angle angles[j] (radians).
 * PAR2D: ray direction (-sin, cos), detector axis (cos, sin); bin k at
 *        (k - (n_u-1)/2) du; n_v must be 1.
 * CONE3D: source sid (cos, sin, 0), detector centre -idd (cos, sin, 0),
 *        detector axes (-sin, cos, 0) and (0, 0, 1); pixel (a, b) at
 *        ((a - (n_u-1)/2) du, (b - (n_v-1)/2) dv); grids up to n = 1290.
 * FAN2D: the in-plane part of CONE3D: source sid (cos, sin), detector
 *        centre -idd (cos, sin), detector axis (-sin, cos), bin a at
 *        (a - (n_u-1)/2) du; n_v must be 1 and sid > 1.4143 (1 + 2/n)
 *        for an n x n grid (the source well outside the image square). */
typedef struct {
    int kind;
    int n_views, n_u, n_v;
    double du, dv;
    double sid, idd;        /* cone and fan only                            */
    const double *angles;   /* HOST array [n_views]                         */
} ct_geometry;

/* INR architectures (Sec. IV names all three).  HASH: the hash encoding of
 * Mueller et al. (2022) with 2 features per level feeding a ReLU MLP.  Level
 * l of Lh has resolution N_l = floor(base_res b^l + 1e-6), b = (max_res /
 * base_res)^(1/(Lh-1)); a point x in [-1,1]^d lies at p = (x+1)/2 N_l; its
 * cell's 2^d vertices c get multilinear weights; vertex c indexes the
 * level's 2^log2_size-entry table densely (sum c_i (N_l+1)^i) when
 * (N_l+1)^d fits, else by the spatial hash (XOR_i c_i pi_i) mod T, pi = (1,
 * 2654435761, 805459861), 32-bit.  Parameters: the tables [Lh][T][2]
 * first, then the MLP (input 2 Lh) in the usual layout.  HASH runs in FP32
 * with width 16, 32 or 64 and width * depth <= 128. */
typedef struct {
    int kind;               /* INRCT_FFN, INRCT_SIREN or INRCT_HASH         */
    int in_dim;             /* d = 2 or 3 (must equal the grid's dim)       */
    int n_freq;             /* FFN: F (encoding width 2F, F % 8 == 0)       */
    int width;              /* hidden width: 128 or 256 (HASH: 16, 32, 64)  */
    int depth;              /* hidden layers L (1..8; HASH 1..4)            */
    float omega0;           /* SIREN frequency factor                       */
    int mlp_dtype;          /* INRCT_FP32 or INRCT_BF16 (HASH: FP32)        */
    int hash_levels;        /* HASH: Lh, 1..32                              */
    int hash_log2_size;     /* HASH: log2 T, 4..24                          */
    int hash_base_res;      /* HASH: N_0 >= 1                               */
    int hash_max_res;       /* HASH: N_{Lh-1} >= N_0                        */
} inr_arch;

typedef struct inrct_geom inrct_geom;
typedef struct inrct_model inrct_model;
typedef struct inr_ctx inr_ctx;

/* Message for the most recent error on this thread ("" if none). */
const char *inrct_last_error(void);

/* workspace kinds */
#define INRCT_WS_GEOM 1     /* inrct_geom_create: needs g, grid             */
#define INRCT_WS_MODEL 2    /* inrct_model_create: needs arch, grid, max_k  */
#define INRCT_WS_CTX 3      /* inr_ctx_create: arch, g, grid, max_k, cfg    */

typedef struct inrct_step_cfg inrct_step_cfg;

/* Exact device bytes the workspace of a handle needs: the geometry handle
 * of (g, grid), the model handle of (arch, grid, max_k), or the context of
 * such a model and geometry with step configuration cfg.  Arguments a kind
 * does not use may be NULL.  Runs only host arithmetic (the handle's build
 * code in a counting mode), so a caller can budget device memory before
 * creating anything.  Returns the byte count, or a negative status with
 * the same argument checks as the create call. */
int64_t inrct_workspace_bytes(int which, const inr_arch *arch,
                              const ct_geometry *g, const inr_grid *grid,
                              int64_t max_k, const inrct_step_cfg *cfg);

/* ------------------------------------------------------------------ P, P^T
 * Joseph's ray-driven projector (Sec. III: P in R^{m x n}, a discrete
 * approximation of ray integrals).  Per ray: one sample per grid slice
 * along the principal axis (y if |d_y| >= (1 - 1e-9)|d_x|, else x; decided
 * in float64 on the host), linear (2D) or bilinear (3D) interpolation with
 * zero padding at fractional index (q + 1)/h - 1/2, times the step length
 * h |d| / |d_axis|.  Interpolation positions are stepped in 32.32 fixed
 * point from float64 ray parameters, so P and P^T see identical weights.
 */

/* Builds the geometry tables (host float64) and uploads them into the
 * handle's workspace (see the conventions above; size from
 * inrct_workspace_bytes(INRCT_WS_GEOM, ...)).  `g` and `grid` are copied.
 * CONE3D fails with INRCT_EINVAL if any detector row is steeper in z than
 * along its ray's in-plane principal axis. */
int inrct_geom_create(const ct_geometry *g, const inr_grid *grid, void *ws,
                      size_t ws_bytes, hipStream_t stream, inrct_geom **out);
int inrct_geom_destroy(inrct_geom *geom);
/* number of rays m = n_views * n_v * n_u */
int64_t inrct_geom_n_rays(const inrct_geom *geom);

/* Which adjoint formulation ct_backproject uses for this geometry (chosen
 * when the geometry is built; every form computes the same v = P^T r up to
 * FP32 summation order): INRCT_ADJ_2D (parallel or fan beam),
 * INRCT_ADJ_DIRECT (cone, gathers from global memory), INRCT_ADJ_WALK (cone,
 * detector footprints staged in LDS, row walk per voxel column),
 * INRCT_ADJ_WALK2 (the same, rows half a voxel to a voxel apart: two rows
 * per voxel band, no branch).  -1 for a null handle. */
#define INRCT_ADJ_2D 0
#define INRCT_ADJ_DIRECT 1
#define INRCT_ADJ_WALK 2
#define INRCT_ADJ_WALK2 3
int inrct_geom_adjoint_kind(const inrct_geom *geom);

/* z = P u.  u: device [grid], z: device [rays].  The whole grid is
 * integrated (values outside the FOV count). */
int ct_project(inrct_geom *geom, const float *u, float *z, hipStream_t stream);

/* v = P^T r, the exact transpose of ct_project (Sec. III, v = P^T r),
 * evaluated voxel by voxel as a gather over the rays whose interpolation
 * stencil touches the voxel (no atomics).  r: device [rays]; v: device
 * [grid], every grid point written. */
int ct_backproject(inrct_geom *geom, const float *r, float *v,
                   hipStream_t stream);

/* v_I = (P^T r)_i for the k grid indices idx (device int32); v_out device
 * [k].  Same arithmetic as ct_backproject at those voxels. */
int ct_backproject_at(inrct_geom *geom, const float *r, const int32_t *idx,
                      int64_t k, float *v_out, hipStream_t stream);

/* r = dL/dz and L (Sec. II; Sec. III note after Algorithm 1).
 * loss == INRCT_LS: r = z - y, L = 1/2 sum r^2.
 * loss == INRCT_FLS: q = z - y, r = F q with F the Ram-Lak ramp along the
 * detector-u index of every (view, row) (linear convolution, taps
 * f0 = 1/(4 du), f_j = -1/(pi^2 j^2 du) for odd j), L = 1/2 q.r.
 * z, y, r: device [rays] (r may alias z); loss_out: device double,
 * accumulated in float64 with a fixed-order reduction. */
int inrct_residual_loss(inrct_geom *geom, int loss, const float *z,
                        const float *y, float *r, double *loss_out,
                        hipStream_t stream);

/* ------------------------------------------------------------------ E, VJP
 * INR f_theta (Sec. IV: FFN and SIREN) evaluated with matrix-core GEMMs.
 * `max_k` bounds the k of later inr_vjp_subsampled / inrct_sample calls
 * (it sizes the handle's scratch; workspace from
 * inrct_workspace_bytes(INRCT_WS_MODEL, ...)).  `arch` and `grid` are
 * copied. */
int inrct_model_create(const inr_arch *arch, const inr_grid *grid,
                       int64_t max_k, void *ws, size_t ws_bytes,
                       hipStream_t stream, inrct_model **out);
int inrct_model_destroy(inrct_model *model);
int64_t inrct_model_n_params(const inrct_model *model);
int64_t inrct_model_n_fov(const inrct_model *model);

/* u = E{f_theta} (Sec. III): f_theta at every FOV point, 0 elsewhere, no
 * autodiff state kept.  theta: device [p]; B: device [F][d] (FFN) or NULL;
 * u: device [grid]. */
int inr_eval_grid(inrct_model *model, const float *theta, const float *B,
                  float *u, hipStream_t stream);

/* f_theta at k grid points idx (device int32) -> f_out device [k]. */
int inr_eval_points(inrct_model *model, const float *theta, const float *B,
                    const int32_t *idx, int64_t k, float *f_out,
                    hipStream_t stream);

/* grad = scale * sum_{j<k} v_j grad_theta f_theta(x_{idx_j}) -- Eq. (2)
 * with scale = n/|I|, equivalently the gradient of the virtual loss of
 * Eq. (3).  Layer activations are recomputed per tile of points and never
 * stored for the whole set.  v: device; if v_compact is 0 it is a full
 * grid indexed by idx, else it holds the k values v_{idx_j} in order.
 * grad: device [p], overwritten. */
int inr_vjp_subsampled(inrct_model *model, const float *theta,
                       const float *B, const int32_t *idx, int64_t k,
                       const float *v, int v_compact, double scale,
                       float *grad, hipStream_t stream);

/* I (Algorithm 1, "sample random index set"): the first k images of the
 * keyed pseudo-random permutation pi_{seed,step} of the FOV ranks [0, n),
 * sorted, as grid indices.  pi: SplitMix64-keyed 6-round Feistel network
 * on 2*hb bits (2^(2hb) >= n, hb = ceil(b/2), b = max(2, ceil(log2 n)))
 * with cycle walking; round key K_r = mix64(seed ^ mix64(step ^
 * (0x9E3779B97F4A7C15 (r+1)))), round function mix64(K_r ^ R) >> (64 -
 * hb).  idx_out: device int32 [k]; 1 <= k <= min(n, max_k). */
int inrct_sample(inrct_model *model, uint64_t seed, uint64_t step, int64_t k,
                 int32_t *idx_out, hipStream_t stream);

/* Adam (Kingma & Ba; the paper's optimiser, Sec. IV) with bias correction,
 * t the 1-based step.  theta, m, v, g: device [p]; theta, m, v updated in
 * place.  gnorm2_out: device double, ||g||^2 reduced in float64 (may be
 * NULL). */
int inrct_adam(inrct_model *model, float *theta, float *m, float *v,
               const float *g, int64_t t, double lr, double beta1,
               double beta2, double eps, double *gnorm2_out,
               hipStream_t stream);

/* Adam as inrct_adam (same kernels, bitwise the same theta, m, v and
 * ||g||^2), without a model handle or workspace, for callers that cannot
 * allocate device memory: code under HIP graph capture, tight serving
 * loops, harnesses that forbid hipMalloc.  The float64 partials of ||g||^2
 * live in a static device array of 1024 doubles (8 KB) that each GPU the
 * library runs on keeps until the process ends; its address is looked up
 * once per device on the first call there.  p: parameters, 1 <=
 * p <= INRCT_ADAM_NOALLOC_MAX_P (any p needs at most those 1024 partials);
 * a larger p is refused with INRCT_EINVAL.  Every partial the reduction
 * reads is written by the same call first, so nothing carries over between
 * calls; but calls that overlap on one device (different streams, or
 * different threads) share the array and race.  Allocates nothing. */
#define INRCT_ADAM_NOALLOC_MAX_P 2147483647LL
int inrct_adam_noalloc(float *theta, float *m, float *v, const float *g,
                       int64_t p, int64_t t, double lr, double beta1,
                       double beta2, double eps, double *gnorm2_out,
                       hipStream_t stream);

/* ------------------------------------------------------------ full step */
struct inrct_step_cfg {
    int loss;               /* INRCT_LS or INRCT_FLS                        */
    int64_t k;              /* |I|; k == n is full sampling                 */
    uint64_t seed;          /* sampler key                                  */
    double lr, beta1, beta2, eps;
    int v_mode;             /* INRCT_V_FULL or INRCT_V_AT_I                 */
};

/* A context binds a model, a geometry and caller-owned device buffers
 * theta [p], adam_m [p], adam_v [p], B [F][d] (or NULL) and y [rays].  Its
 * own u, z/r, v, g and I buffers live in its workspace
 * (inrct_workspace_bytes(INRCT_WS_CTX, ...)); u outside the FOV is cleared
 * on `stream`. */
int inr_ctx_create(inrct_model *model, inrct_geom *geom,
                   const inrct_step_cfg *cfg, float *theta, float *adam_m,
                   float *adam_v, const float *B, const float *y, void *ws,
                   size_t ws_bytes, hipStream_t stream, inr_ctx **out);
int inr_ctx_destroy(inr_ctx *ctx);

/* One Algorithm-1 gradient estimate followed by one Adam update, all on
 * `stream`: u = E f; z = P u; r, L; v = P^T r; I = sample(seed, step);
 * g = (n/k) sum_I v_i grad f(x_i); theta <- Adam(theta, g) with t =
 * step + 1.  loss_out, gnorm2_out: device doubles (L at the incoming theta
 * and ||g||^2), either may be NULL. */
int inr_grad_step(inr_ctx *ctx, uint64_t step, double *loss_out,
                  double *gnorm2_out, hipStream_t stream);

/* The same step with the loss restricted to a subset of the views (the
 * ordered-subsets use of Algorithm 1 noted at the end of Sec. III): P, the
 * residual and P^T use `geom` and `y` in place of the context's geometry
 * and data; everything else is inr_grad_step's.  The loss is the subset's
 * own, 1/2 ||P_S u - y_S||^2 (LS) or its FLS form, not rescaled.  geom:
 * any geometry on the context's grid with at most as many rays as the
 * context's geometry (typically the context geometry's views j with
 * j mod S == s, built from those angles); y: device float [rays of geom],
 * in geom's ray order.  Caller keeps ownership of both. */
int inr_grad_step_views(inr_ctx *ctx, uint64_t step, inrct_geom *geom,
                        const float *y, double *loss_out, double *gnorm2_out,
                        hipStream_t stream);

/* Stage timing with HIP events recorded on the step's stream, for
 * measurement.  After inr_ctx_enable_timing(ctx, max_steps), each
 * inr_grad_step records events around its stages (slots reused modulo
 * max_steps).  inr_ctx_stage_ms waits for the recorded events, writes the
 * summed milliseconds of stages 0..n_stages-1 over the recorded steps and
 * starts a new recording.  Stages: 0 grid-evaluation kernel, 1 P, 2
 * residual, 3 sampler, 4 P^T, 5 VJP, 6 Adam, 7 whole step. */
int inr_ctx_enable_timing(inr_ctx *ctx, int max_steps);
int inr_ctx_stage_ms(inr_ctx *ctx, int n_stages, double *ms_out);

/* Device buffers owned by the context (valid until inr_ctx_destroy), for
 * inspection: which = 0 u [grid], 1 r [rays], 2 v [grid or k], 3 g [p],
 * 4 I [k] (int32). */
void *inr_ctx_buffer(inr_ctx *ctx, int which);

#ifdef __cplusplus
}
#endif
#endif /* INRCT_H */
