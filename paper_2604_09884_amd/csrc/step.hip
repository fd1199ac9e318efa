// Index sampler, Adam, and Algorithm 1 + Adam on a context.
//
// Sampler: the first k images of a keyed pseudo-random permutation of the
// FOV ranks (a uniform k-subset without replacement, so Eq. (2) is
// unbiased).  Marks are written into a byte per FOV rank -- each rank is
// hit by exactly one thread because the map is a bijection -- and compacted
// in rank order with a fixed-order scan, giving sorted grid indices.
#include <math.h>

#include <map>
#include <mutex>

#include "model.h"

namespace inrct {

// --------------------------------------------------------------- sampler
__device__ __forceinline__ unsigned long long mix64(unsigned long long z) {
    z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ULL;
    z = (z ^ (z >> 27)) * 0x94D049BB133111EBULL;
    return z ^ (z >> 31);
}

struct PrpKey {
    unsigned long long k[6];
    int hb;
    unsigned long long n;
};

static PrpKey make_key(uint64_t seed, uint64_t step, long long n) {
    auto hmix = [](unsigned long long z) {
        z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ULL;
        z = (z ^ (z >> 27)) * 0x94D049BB133111EBULL;
        return z ^ (z >> 31);
    };
    PrpKey key;
    int b = 2;
    while ((1ULL << b) < (unsigned long long)n) ++b;
    key.hb = (b + 1) / 2;
    key.n = (unsigned long long)n;
    for (int r = 0; r < 6; ++r)
        key.k[r] = hmix(seed ^ hmix(step ^ (0x9E3779B97F4A7C15ULL * (unsigned long long)(r + 1))));
    return key;
}

__device__ __forceinline__ unsigned long long feistel(unsigned long long x, const PrpKey &key) {
    const int hb = key.hb;
    const unsigned long long mask = (1ULL << hb) - 1;
    unsigned long long L = x >> hb, R = x & mask;
#pragma unroll
    for (int r = 0; r < 6; ++r) {
        const unsigned long long t = L ^ (mix64(key.k[r] ^ R) >> (64 - hb));
        L = R;
        R = t;
    }
    return (L << hb) | R;
}

// flags[pi(j)] = 1 for j < k.  Cycle walking ends because the orbit of j
// under the bijection returns to j < n; the bound is a guard only.
__global__ void k_mark(PrpKey key, long long k, unsigned char *__restrict__ flags,
                       int *__restrict__ overflow) {
    const long long j = (long long)blockIdx.x * 256 + threadIdx.x;
    if (j >= k) return;
    unsigned long long y = feistel((unsigned long long)j, key);
    const unsigned long long dom = 1ULL << (2 * key.hb);
    unsigned long long it = 0;
    while (y >= key.n && it < dom) {
        y = feistel(y, key);
        ++it;
    }
    if (y < key.n) flags[y] = 1;
    else overflow[0] = 1;
}

// per-block counts of set flags (4096 flags per block, 256 threads x 16)
// Flags set among ranks [base, base + 16): one 16-byte load when the run
// lies inside [0, n) (base is a multiple of 16, the array 256-byte
// aligned), else byte by byte.
__device__ __forceinline__ int count16(const unsigned char *__restrict__ flags, long long base,
                                       long long n) {
    if (base + 16 <= n) {
        const uint4 w = *(const uint4 *)(flags + base);
        // each byte is 0 or 1: the byte sum of a word is its count
        auto bytes = [](unsigned x) { return (int)((x * 0x01010101u) >> 24); };
        return bytes(w.x) + bytes(w.y) + bytes(w.z) + bytes(w.w);
    }
    int c = 0;
    for (int i = 0; i < 16; ++i)
        if (base + i < n) c += flags[base + i];
    return c;
}

__global__ __launch_bounds__(256) void k_count(const unsigned char *__restrict__ flags,
                                               long long n, long long *__restrict__ blk) {
    __shared__ int sh[256];
    const long long base = (long long)blockIdx.x * 4096 + threadIdx.x * 16;
    const int c = count16(flags, base, n);
    sh[threadIdx.x] = c;
    __syncthreads();
    for (int s = 128; s > 0; s >>= 1) {
        if (threadIdx.x < s) sh[threadIdx.x] += sh[threadIdx.x + s];
        __syncthreads();
    }
    if (threadIdx.x == 0) blk[blockIdx.x] = sh[0];
}

// exclusive scan of the block counts, in place (single block of 1024)
__global__ __launch_bounds__(1024) void k_scan(long long *__restrict__ blk, long long nb) {
    __shared__ long long sh[1024];
    const int t = threadIdx.x;
    const long long per = (nb + 1023) / 1024;
    const long long lo = t * per, hi = lo + per < nb ? lo + per : nb;
    long long s = 0;
    for (long long i = lo; i < hi; ++i) s += blk[i];
    sh[t] = s;
    __syncthreads();
    for (int off = 1; off < 1024; off <<= 1) {  // inclusive Hillis-Steele
        long long v = t >= off ? sh[t - off] : 0;
        __syncthreads();
        sh[t] += v;
        __syncthreads();
    }
    long long run = sh[t] - s;
    for (long long i = lo; i < hi; ++i) {
        const long long c = blk[i];
        blk[i] = run;
        run += c;
    }
}

__global__ __launch_bounds__(256) void k_emit(const unsigned char *__restrict__ flags, long long n,
                                              const long long *__restrict__ blk, FovDev fov,
                                              int32_t *__restrict__ out) {
    __shared__ int sh[256];
    const long long base = (long long)blockIdx.x * 4096 + threadIdx.x * 16;
    const int c = count16(flags, base, n);
    sh[threadIdx.x] = c;
    __syncthreads();
    for (int off = 1; off < 256; off <<= 1) {
        int v = threadIdx.x >= off ? sh[threadIdx.x - off] : 0;
        __syncthreads();
        sh[threadIdx.x] += v;
        __syncthreads();
    }
    long long pos = blk[blockIdx.x] + sh[threadIdx.x] - c;
    if (c == 0) return;
    // the row of the first set rank by binary search, later ones by walking
    // forward (16 consecutive ranks cross at most a few row starts)
    bool found = false;
    int z = 0, y = 0;
    long long zbase = 0;
    for (int i = 0; i < 16; ++i) {
        const long long q = base + i;
        if (q >= n || !flags[q]) continue;
        if (!found) {
            int x;
            out[pos++] = (int32_t)fov_rank_to_index(fov, q, &x, &y, &z);
            zbase = (long long)z * fov.n_slice;
            found = true;
            continue;
        }
        long long rem = q - zbase;
        while (rem >= fov.n_slice) {  // next z slice
            ++z;
            zbase += fov.n_slice;
            rem -= fov.n_slice;
            y = 0;
        }
        while (y + 1 < fov.N && fov.row_start[y + 1] <= rem) ++y;
        const int x = fov.xlo[y] + (int)(rem - fov.row_start[y]);
        out[pos++] = (int32_t)(((long long)z * fov.N + y) * fov.N + x);
    }
}

void model_sample(inrct_model *m, uint64_t seed, uint64_t step, long long k, int32_t *idx,
                  hipStream_t s) {
    const long long n = m->n_fov;
    const PrpKey key = make_key(seed, step, n);
    launch_zero_bytes(m->flags.ptr, (size_t)n, s);
    // the overflow word lives after the block counts (never set in practice)
    hipLaunchKernelGGL(k_mark, dim3((unsigned)cdiv(k, 256)), dim3(256), 0, s, key, k,
                       m->flags.as<unsigned char>(),
                       (int *)(m->blk.as<long long>() + m->n_blk));
    INRCT_CHECK_LAUNCH();
    hipLaunchKernelGGL(k_count, dim3((unsigned)m->n_blk), dim3(256), 0, s,
                       m->flags.as<unsigned char>(), n, m->blk.as<long long>());
    INRCT_CHECK_LAUNCH();
    hipLaunchKernelGGL(k_scan, dim3(1), dim3(1024), 0, s, m->blk.as<long long>(), m->n_blk);
    INRCT_CHECK_LAUNCH();
    hipLaunchKernelGGL(k_emit, dim3((unsigned)m->n_blk), dim3(256), 0, s,
                       m->flags.as<unsigned char>(), n, m->blk.as<long long>(),
                       m->fov.dev(m->dim), idx);
    INRCT_CHECK_LAUNCH();
}

// ------------------------------------------------------------------ Adam
__global__ __launch_bounds__(256) void k_adam(float *__restrict__ th, float *__restrict__ mm,
                                              float *__restrict__ vv, const float *__restrict__ g,
                                              long long p, float b1, float b2, float step_size,
                                              float inv_sqrt_bc2, float eps,
                                              double *__restrict__ partials) {
    __shared__ double sh[256];
    double acc = 0.0;
    const long long stride = (long long)gridDim.x * 256;
    for (long long i = (long long)blockIdx.x * 256 + threadIdx.x; i < p; i += stride) {
        const float gi = g[i];
        const float mi = b1 * mm[i] + (1.f - b1) * gi;
        const float vi = b2 * vv[i] + (1.f - b2) * gi * gi;
        mm[i] = mi;
        vv[i] = vi;
        th[i] -= step_size * mi / (sqrtf(vi) * inv_sqrt_bc2 + eps);
        acc += (double)gi * (double)gi;
    }
    const double s = block_sum_f64(acc, sh);
    if (threadIdx.x == 0) partials[blockIdx.x] = s;
}

// Blocks of the Adam launch for p parameters: one float64 partial of ||g||^2
// each, at most kAdamMaxPartials.
int adam_partials(long long p) {
    return (int)std::min<long long>(kAdamMaxPartials, std::max<long long>(1, cdiv(p, 2048)));
}

// Adam over p parameters with the partials of ||g||^2 in `partials` (at
// least adam_partials(p) doubles).
static void launch_adam(float *theta, float *mm, float *vv, const float *g, long long p,
                        long long t, double lr, double b1, double b2, double eps, double *gn2,
                        double *partials, hipStream_t s) {
    const double bc1 = 1.0 - pow(b1, (double)t);
    const double bc2 = 1.0 - pow(b2, (double)t);
    const int nb = adam_partials(p);
    hipLaunchKernelGGL(k_adam, dim3(nb), dim3(256), 0, s, theta, mm, vv, g, p, (float)b1,
                       (float)b2, (float)(lr / bc1), (float)(1.0 / sqrt(bc2)), (float)eps,
                       partials);
    INRCT_CHECK_LAUNCH();
    if (gn2) launch_sum_partials(partials, nb, gn2, s);
}

void model_adam(inrct_model *m, float *theta, float *mm, float *vv, const float *g, long long t,
                double lr, double b1, double b2, double eps, double *gn2, hipStream_t s) {
    launch_adam(theta, mm, vv, g, m->n_params, t, lr, b1, b2, eps, gn2, m->apart.as<double>(),
                s);
}

// ---------------------------------------------- Adam without allocation
// The float64 partials of inrct_adam_noalloc live in this file-scope device
// array (each device the library runs on holds its own copy until the
// process ends).  Host code never passes the array's name to a kernel: the
// name is a host-side stand-in, not a device address.  The address comes
// from hipGetSymbolAddress, once per device, with that device current.
static __device__ __align__(256) double scratch[kAdamMaxPartials];

static double *scratch_ptr() {
    static std::mutex mu;
    static std::map<int, double *> ptrs;
    int dev = 0;
    INRCT_CHECK_HIP(hipGetDevice(&dev));
    std::lock_guard<std::mutex> lock(mu);
    auto it = ptrs.find(dev);
    if (it != ptrs.end()) return it->second;
    void *p = nullptr;
    INRCT_CHECK_HIP(hipGetSymbolAddress(&p, HIP_SYMBOL(scratch)));
    INRCT_REQUIRE(p != nullptr, "no device address for the Adam scratch array");
    ptrs[dev] = (double *)p;
    return (double *)p;
}

}  // namespace inrct

// ==================================================================== ABI
using namespace inrct;

struct inr_ctx {
    inrct::Workspace ws;
    inrct_model *model = nullptr;
    inrct_geom *geom = nullptr;
    inrct_step_cfg cfg;
    float *theta = nullptr, *am = nullptr, *av = nullptr;
    const float *B = nullptr, *y = nullptr;
    int64_t m_cap = 0;  // rays the r buffer holds
    DevBuf u, r, v, g, idx;
    DevBuf ut;  // cone beam: u transposed in every xy plane ([z][x][y])
    // optional stage timing: events[slot][stage][0=start, 1=end]
    std::vector<hipEvent_t> events;
    int t_slots = 0, t_used = 0;
    ~inr_ctx() {
        for (hipEvent_t e : events) (void)hipEventDestroy(e);
    }
    hipEvent_t ev(int stage, int end) const {
        const int slot = t_used % t_slots;
        return events[((size_t)slot * kStages + stage) * 2 + end];
    }
    static const int kStages = 8;
};

namespace inrct {
// The context's own buffers: u and v on the grid (v only at I when v_mode
// is INRCT_V_AT_I), r on the rays, g, and I; for a cone geometry also the
// plane-wise transpose of u that the x-principal rays read.  u outside the
// FOV is 0 and no step writes there, so it is cleared once here.
static void build_ctx(inr_ctx *c, long long n_grid, long long m_rays, long long n_params,
                      bool cone, Arena &ar) {
    c->m_cap = m_rays;
    c->u.alloc(ar, sizeof(float) * n_grid);
    zero_fill(ar, c->u);
    if (cone) {
        c->ut.alloc(ar, sizeof(float) * n_grid);
        zero_fill(ar, c->ut);
    }
    c->r.alloc(ar, sizeof(float) * m_rays);
    c->v.alloc(ar, sizeof(float) * (c->cfg.v_mode == INRCT_V_FULL ? n_grid : c->cfg.k));
    c->g.alloc(ar, sizeof(float) * n_params);
    c->idx.alloc(ar, sizeof(int32_t) * c->cfg.k);
}

static void check_cfg(const inrct_step_cfg *cfg, long long max_k) {
    INRCT_REQUIRE(cfg, "null step configuration");
    INRCT_REQUIRE(cfg->k >= 1 && cfg->k <= max_k, "k must be in [1, max_k=%lld]", max_k);
    INRCT_REQUIRE(cfg->loss == INRCT_LS || cfg->loss == INRCT_FLS, "unknown loss");
    INRCT_REQUIRE(cfg->v_mode == INRCT_V_FULL || cfg->v_mode == INRCT_V_AT_I, "unknown v_mode");
    INRCT_REQUIRE(cfg->lr > 0 && cfg->eps > 0 && cfg->beta1 >= 0 && cfg->beta1 < 1 &&
                      cfg->beta2 >= 0 && cfg->beta2 < 1,
                  "bad Adam hyper-parameters");
}
}  // namespace inrct

extern "C" {

int inrct_sample(inrct_model *model, uint64_t seed, uint64_t step, int64_t k, int32_t *idx_out,
                 hipStream_t stream) {
    return guarded([&] {
        INRCT_REQUIRE(model && idx_out, "null argument");
        INRCT_REQUIRE(k >= 1 && k <= model->max_k, "k must be in [1, max_k=%lld]",
                      (long long)model->max_k);
        model_sample(model, seed, step, k, idx_out, stream);
    });
}

int inrct_adam(inrct_model *model, float *theta, float *m, float *v, const float *g, int64_t t,
               double lr, double beta1, double beta2, double eps, double *gnorm2_out,
               hipStream_t stream) {
    return guarded([&] {
        INRCT_REQUIRE(model && theta && m && v && g, "null argument");
        INRCT_REQUIRE(t >= 1, "t is 1-based");
        INRCT_REQUIRE(beta1 >= 0 && beta1 < 1 && beta2 >= 0 && beta2 < 1 && eps > 0 && lr > 0,
                      "bad Adam hyper-parameters");
        model_adam(model, theta, m, v, g, t, lr, beta1, beta2, eps, gnorm2_out, stream);
    });
}

int inrct_adam_noalloc(float *theta, float *m, float *v, const float *g, int64_t p, int64_t t,
                       double lr, double beta1, double beta2, double eps, double *gnorm2_out,
                       hipStream_t stream) {
    return guarded([&] {
        INRCT_REQUIRE(theta && m && v && g, "null argument");
        INRCT_REQUIRE(p >= 1 && p <= INRCT_ADAM_NOALLOC_MAX_P,
                      "p = %lld outside [1, %lld] (the partials array holds %d entries)",
                      (long long)p, (long long)INRCT_ADAM_NOALLOC_MAX_P, kAdamMaxPartials);
        INRCT_REQUIRE(t >= 1, "t is 1-based");
        INRCT_REQUIRE(beta1 >= 0 && beta1 < 1 && beta2 >= 0 && beta2 < 1 && eps > 0 && lr > 0,
                      "bad Adam hyper-parameters");
        // every partial the reduction reads is written by the Adam launch
        // first, so nothing needs clearing between calls
        launch_adam(theta, m, v, g, p, t, lr, beta1, beta2, eps, gnorm2_out, scratch_ptr(),
                    stream);
    });
}

int inr_ctx_create(inrct_model *model, inrct_geom *geom, const inrct_step_cfg *cfg, float *theta,
                   float *adam_m, float *adam_v, const float *B, const float *y, void *ws,
                   size_t ws_bytes, hipStream_t stream, inr_ctx **out) {
    return guarded([&] {
        INRCT_REQUIRE(model && geom && cfg && theta && adam_m && adam_v && y && out,
                      "null argument");
        *out = nullptr;
        INRCT_REQUIRE(geom_dim(geom) == model->dim && geom_N(geom) == model->N,
                      "model grid and geometry grid differ");
        INRCT_REQUIRE(model->arch.kind != INRCT_FFN || B, "FFN needs B");
        check_cfg(cfg, model->max_k);
        auto fresh = [&] {
            inr_ctx *c = new inr_ctx();
            c->cfg = *cfg;
            return c;
        };
        const long long ng = model->n_grid, mr = geom_rays(geom), np = model->n_params;
        const bool cone = geom->g.kind == INRCT_CONE3D;
        inr_ctx *c = fresh();
        try {
            c->model = model;
            c->geom = geom;
            c->theta = theta;
            c->am = adam_m;
            c->av = adam_v;
            c->B = B;
            c->y = y;
            build_in_workspace(c, c->ws, ws, ws_bytes, stream, fresh,
                               [&](inr_ctx *x, Arena &ar) { build_ctx(x, ng, mr, np, cone, ar); });
        } catch (...) {
            delete c;
            throw;
        }
        *out = c;
    });
}

int64_t inrct_workspace_bytes(int which, const inr_arch *arch, const ct_geometry *g,
                              const inr_grid *grid, int64_t max_k, const inrct_step_cfg *cfg) {
    int64_t bytes = 0;
    const int st = guarded([&] {
        if (which == INRCT_WS_GEOM) {
            check_geom_args(g, grid);
            bytes = (int64_t)workspace_need<inrct_geom>(
                [&] { return fresh_geom(g, grid); },
                [](inrct_geom *x, Arena &ar) { build_geom(x, ar); });
        } else if (which == INRCT_WS_MODEL || which == INRCT_WS_CTX) {
            check_model_args(arch, grid, max_k);
            inrct_model *tm = fresh_model(arch, grid, max_k);
            Arena sz;
            try {
                build_model(tm, sz);
            } catch (...) {
                delete tm;
                throw;
            }
            const long long ng = tm->n_grid, np = tm->n_params, kmax = tm->max_k;
            delete tm;
            if (which == INRCT_WS_MODEL) {
                bytes = (int64_t)sz.used;
                return;
            }
            // the context: u, r, v, g and I for this model and geometry
            INRCT_REQUIRE(g, "null geometry");
            check_cfg(cfg, kmax);
            const long long mr = (long long)g->n_views * g->n_u * g->n_v;
            bytes = (int64_t)workspace_need<inr_ctx>(
                [&] {
                    inr_ctx *c = new inr_ctx();
                    c->cfg = *cfg;
                    return c;
                },
                [&](inr_ctx *x, Arena &ar) {
                    build_ctx(x, ng, mr, np, g->kind == INRCT_CONE3D, ar);
                });
        } else {
            set_error("unknown workspace kind %d", which);
            throw Error{INRCT_EINVAL};
        }
    });
    return st == INRCT_OK ? bytes : (int64_t)st;
}

int inr_ctx_destroy(inr_ctx *ctx) {
    delete ctx;
    return INRCT_OK;
}

void *inr_ctx_buffer(inr_ctx *ctx, int which) {
    if (!ctx) return nullptr;
    switch (which) {
        case 0: return ctx->u.ptr;
        case 1: return ctx->r.ptr;
        case 2: return ctx->v.ptr;
        case 3: return ctx->g.ptr;
        case 4: return ctx->idx.ptr;
        default: return nullptr;
    }
}

int inr_ctx_enable_timing(inr_ctx *c, int max_steps) {
    return guarded([&] {
        INRCT_REQUIRE(c && max_steps >= 1 && max_steps <= 100000, "bad arguments");
        for (hipEvent_t e : c->events) (void)hipEventDestroy(e);
        c->events.assign((size_t)max_steps * inr_ctx::kStages * 2, nullptr);
        for (auto &e : c->events) INRCT_CHECK_HIP(hipEventCreate(&e));
        c->t_slots = max_steps;
        c->t_used = 0;
    });
}

int inr_ctx_stage_ms(inr_ctx *c, int n_stages, double *ms_out) {
    return guarded([&] {
        INRCT_REQUIRE(c && ms_out && n_stages >= 1 && n_stages <= inr_ctx::kStages,
                      "bad arguments");
        INRCT_REQUIRE(c->t_slots > 0, "timing not enabled");
        const int steps = std::min(c->t_used, c->t_slots);
        for (int st = 0; st < n_stages; ++st) {
            double tot = 0.0;
            for (int k = 0; k < steps; ++k) {
                float ms = 0.f;
                hipEvent_t a = c->events[((size_t)k * inr_ctx::kStages + st) * 2];
                hipEvent_t b = c->events[((size_t)k * inr_ctx::kStages + st) * 2 + 1];
                INRCT_CHECK_HIP(hipEventSynchronize(b));
                INRCT_CHECK_HIP(hipEventElapsedTime(&ms, a, b));
                tot += ms;
            }
            ms_out[st] = tot;
        }
        c->t_used = 0;
    });
}

}  // extern "C"

// One step with projector `geom` and data `y` (the context's own for the
// plain step, a view subset's for ordered subsets).
static void grad_step(inr_ctx *c, uint64_t step, inrct_geom *geom, const float *y,
                      double *loss_out, double *gnorm2_out, hipStream_t s) {
    const bool timed = c->t_slots > 0;
    auto mark = [&](int stage, int end) {
        if (timed) INRCT_CHECK_HIP(hipEventRecord(c->ev(stage, end), s));
    };
    inrct_model *m = c->model;
    const long long k = c->cfg.k;
    float *u = c->u.as<float>(), *r = c->r.as<float>(), *v = c->v.as<float>();
    int32_t *idx = c->idx.as<int32_t>();
    mark(7, 0);
    // Algorithm 1, step 1: z = P E{f_theta}
    model_pack(m, c->theta, s);
    mark(0, 0);
    model_eval_fov(m, c->theta, c->B, u, s);
    mark(0, 1);
    mark(1, 0);
    // the plane-wise transpose of u only when this geometry's projector reads it
    float *ut = c->ut.ptr && geom_reads_transpose(geom) ? c->ut.as<float>() : nullptr;
    if (ut) transpose_planes(u, ut, m->N, m->N, s);
    project(geom, u, r, s, true, ut);  // u vanishes outside the FOV
    mark(1, 1);
    // step 2: r = dL/dz, v = P^T r
    mark(2, 0);
    residual_loss(geom, c->cfg.loss, r, y, r, loss_out, s);
    mark(2, 1);
    // step 3: the index set I
    mark(3, 0);
    model_sample(m, c->cfg.seed, step, k, idx, s);
    mark(3, 1);
    mark(4, 0);
    if (c->cfg.v_mode == INRCT_V_FULL) {
        backproject(geom, r, v, s);
    } else {
        backproject_at(geom, r, idx, k, v, s);
    }
    mark(4, 1);
    // steps 4-5: gradient of the virtual loss, Eq. (2)/(3)
    const double scale = (double)m->n_fov / (double)k;
    mark(5, 0);
    model_vjp(m, c->theta, c->B, idx, k, v, c->cfg.v_mode == INRCT_V_AT_I ? 1 : 0, scale,
              c->g.as<float>(), s, false);
    mark(5, 1);
    mark(6, 0);
    model_adam(m, c->theta, c->am, c->av, c->g.as<float>(), (long long)step + 1, c->cfg.lr,
               c->cfg.beta1, c->cfg.beta2, c->cfg.eps, gnorm2_out, s);
    mark(6, 1);
    mark(7, 1);
    if (timed) ++c->t_used;
}

extern "C" {

int inr_grad_step(inr_ctx *c, uint64_t step, double *loss_out, double *gnorm2_out,
                  hipStream_t s) {
    return guarded([&] {
        INRCT_REQUIRE(c, "null context");
        grad_step(c, step, c->geom, c->y, loss_out, gnorm2_out, s);
    });
}

int inr_grad_step_views(inr_ctx *c, uint64_t step, inrct_geom *geom, const float *y,
                        double *loss_out, double *gnorm2_out, hipStream_t s) {
    return guarded([&] {
        INRCT_REQUIRE(c && geom && y, "null argument");
        INRCT_REQUIRE(geom_dim(geom) == c->model->dim && geom_N(geom) == c->model->N,
                      "geometry grid differs from the context's");
        INRCT_REQUIRE(geom_rays(geom) <= c->m_cap,
                      "geometry has %lld rays, the context holds %lld",
                      (long long)geom_rays(geom), (long long)c->m_cap);
        grad_step(c, step, geom, y, loss_out, gnorm2_out, s);
    });
}

}  // extern "C"
