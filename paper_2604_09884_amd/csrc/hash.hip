// The hash-encoding INR (the third architecture of Sec. IV): the
// multi-resolution hash encoding of Mueller et al. (2022) feeding a small
// ReLU MLP, in FP32.  E and the Eq. (2) VJP for it.
//
// E: one thread per point; the encoding is folded straight into the first
// layer (each level's two interpolated features are multiplied into the
// layer-1 sums as soon as they are formed), hidden activations stay in
// registers and the weights are uniform across the wave (scalar loads).
//
// VJP: one thread per sampled point recomputes the forward pass, runs the
// backward pass and stores its layer inputs and deltas as a point-major row;
// dW then comes from fixed-order sums over slices of points and a
// fixed-order sum of the slices.  The tables' gradient is a sum over (point,
// level, cell vertex) contributions: they are sorted by table entry with a
// stable radix sort (equal entries keep the points' order) and each entry's
// run is summed in order.  No atomics: results are bitwise repeatable.
#include <hipcub/hipcub.hpp>

#include "model.h"

namespace inrct {

struct HashDev {
    const float *theta;
    FovDev fov;
    int N, dim, levels, T, W, L, K;
    int res[kHashMaxLevels];
    int dense[kHashMaxLevels];
    long long loff[kHashMaxDepth + 2];  // MLP layer offsets 1..L+1
};

// Vertex base and fraction of grid coordinate i (pixel centre) at a level
// of resolution R: p = (2i + 1) R / (2N), exactly in integers.
__device__ __forceinline__ void hash_axis(int i, int N, int R, int *c, float *f) {
    const long long num = (long long)(2 * i + 1) * R;
    const long long den = 2LL * N;
    const long long b = num / den;
    *c = (int)b;
    *f = (float)(num - b * den) / (float)den;
}

__device__ __forceinline__ unsigned hash_index(const HashDev &h, int l, int cx, int cy,
                                               int cz) {
    const unsigned R1 = (unsigned)h.res[l] + 1u;
    if (h.dense[l]) return (unsigned)cx + R1 * ((unsigned)cy + R1 * (unsigned)cz);
    const unsigned v = (unsigned)cx ^ ((unsigned)cy * 2654435761u) ^ ((unsigned)cz * 805459861u);
    return v & (unsigned)(h.T - 1);
}

// The two interpolated features of level l at grid point (ix, iy, iz); if
// vidx is given, also the cell's vertex indices and weights (vw).
// The 2^DIM table reads are issued together, then combined in vertex order.
template <int DIM>
__device__ __forceinline__ float2 hash_level(const HashDev &h, int l, int ix, int iy, int iz,
                                             unsigned *vidx, float *vw) {
    constexpr int NV = 1 << DIM;
    int cx, cy, cz = 0;
    float fx, fy, fz = 0.f;
    hash_axis(ix, h.N, h.res[l], &cx, &fx);
    hash_axis(iy, h.N, h.res[l], &cy, &fy);
    if (DIM == 3) hash_axis(iz, h.N, h.res[l], &cz, &fz);
    const float2 *tab = (const float2 *)(h.theta + (size_t)l * h.T * 2);
    unsigned id[NV];
    float2 t[NV];
#pragma unroll
    for (int m = 0; m < NV; ++m) {
        id[m] = hash_index(h, l, cx + (m & 1), cy + ((m >> 1) & 1), cz + ((m >> 2) & 1));
        t[m] = tab[id[m]];
    }
    float2 e = make_float2(0.f, 0.f);
#pragma unroll
    for (int m = 0; m < NV; ++m) {
        const int bx = m & 1, by = (m >> 1) & 1, bz = (m >> 2) & 1;
        const float w = (bx ? fx : 1.f - fx) * (by ? fy : 1.f - fy) *
                        (DIM == 3 ? (bz ? fz : 1.f - fz) : 1.f);
        e.x += w * t[m].x;
        e.y += w * t[m].y;
        if (vidx) {
            vidx[m] = id[m];
            vw[m] = w;
        }
    }
    return e;
}

__device__ __forceinline__ void hash_point(const HashDev &h, long long q, int mode,
                                           const int32_t *idx, int *ix, int *iy, int *iz,
                                           long long *g) {
    if (mode == 0) {
        *g = fov_rank_to_index(h.fov, q, ix, iy, iz);
    } else {
        const long long gi = idx[q];
        *g = gi;
        *ix = (int)(gi % h.N);
        *iy = (int)((gi / h.N) % h.N);
        *iz = (int)(gi / ((long long)h.N * h.N));
    }
}

// Forward to the last hidden layer; acts[l] = a_{l+1}.  If enc is given,
// the encoding a_0 is written there (K floats).
template <int W, int LMAX, int DIM>
__device__ __forceinline__ void hash_forward(const HashDev &h, int ix, int iy, int iz,
                                             float (&acts)[LMAX][W], float *enc) {
    const float *W1 = h.theta + h.loff[1];
    float z[W];
#pragma unroll
    for (int i = 0; i < W; ++i) z[i] = W1[(size_t)W * h.K + i];
    for (int l = 0; l < h.levels; ++l) {
        const float2 e = hash_level<DIM>(h, l, ix, iy, iz, nullptr, nullptr);
        if (enc) {
            enc[2 * l] = e.x;
            enc[2 * l + 1] = e.y;
        }
#pragma unroll
        for (int i = 0; i < W; ++i)
            z[i] += W1[(size_t)i * h.K + 2 * l] * e.x + W1[(size_t)i * h.K + 2 * l + 1] * e.y;
    }
#pragma unroll
    for (int i = 0; i < W; ++i) acts[0][i] = fmaxf(z[i], 0.f);
#pragma unroll
    for (int l = 1; l < LMAX; ++l) {
        if (l >= h.L) break;
        const float *Wl = h.theta + h.loff[l + 1];
#pragma unroll
        for (int i = 0; i < W; ++i) {
            float s = Wl[W * W + i];
#pragma unroll
            for (int j = 0; j < W; ++j) s += Wl[i * W + j] * acts[l - 1][j];
            acts[l][i] = fmaxf(s, 0.f);
        }
    }
}

template <int W, int LMAX, int DIM>
__global__ __launch_bounds__(256) void k_hash_eval(HashDev h, long long n, int mode,
                                                   const int32_t *__restrict__ idx,
                                                   float *__restrict__ out) {
    const long long q = (long long)blockIdx.x * 256 + threadIdx.x;
    if (q >= n) return;
    int ix, iy, iz;
    long long g;
    hash_point(h, q, mode, idx, &ix, &iy, &iz, &g);
    float acts[LMAX][W];
    hash_forward<W, LMAX, DIM>(h, ix, iy, iz, acts, nullptr);
    const float *Wo = h.theta + h.loff[h.L + 1];
    float f = Wo[W];
    for (int l = 0; l < LMAX; ++l)
        if (l == h.L - 1) {
#pragma unroll
            for (int j = 0; j < W; ++j) f += Wo[j] * acts[l][j];
        }
    out[mode == 0 ? g : q] = f;
}

// Row of point t (R floats): a_0 (K) | a_1..a_L (W each) | d_1..d_L (W each)
// | d_out.  Contributions of point t: (level, vertex) keys and the two
// weighted feature gradients.
template <int W, int LMAX, int DIM>
__global__ __launch_bounds__(256) void k_hash_vjp(HashDev h, const int32_t *__restrict__ idx,
                                                  long long k, const float *__restrict__ v,
                                                  int v_compact, float scale,
                                                  float *__restrict__ rows, int R,
                                                  uint32_t *__restrict__ ckey,
                                                  uint32_t *__restrict__ cpos,
                                                  float2 *__restrict__ cval) {
    const long long t = (long long)blockIdx.x * 256 + threadIdx.x;
    if (t >= k) return;
    int ix, iy, iz;
    long long g;
    hash_point(h, t, 1, idx, &ix, &iy, &iz, &g);
    float *row = rows + (size_t)t * R;
    float acts[LMAX][W];
    hash_forward<W, LMAX, DIM>(h, ix, iy, iz, acts, row);
    const int K = h.K, L = h.L;
#pragma unroll
    for (int l = 0; l < LMAX; ++l)
        if (l < L) {
#pragma unroll
            for (int i = 0; i < W; ++i) row[K + l * W + i] = acts[l][i];
        }
    const float c = scale * (v_compact ? v[t] : v[g]);
    row[K + 2 * L * W] = c;
    // backward: ga = dL/da_l, gz = dL/dz_l
    const float *Wo = h.theta + h.loff[L + 1];
    float ga[W], gz[W];
#pragma unroll
    for (int i = 0; i < W; ++i) ga[i] = c * Wo[i];
#pragma unroll
    for (int l = LMAX - 1; l >= 0; --l) {
        if (l >= L) continue;
#pragma unroll
        for (int i = 0; i < W; ++i) {
            gz[i] = acts[l][i] > 0.f ? ga[i] : 0.f;
            row[K + L * W + l * W + i] = gz[i];
        }
        if (l > 0) {
            const float *Wl = h.theta + h.loff[l + 1];
#pragma unroll
            for (int j = 0; j < W; ++j) {
                float s = 0.f;
#pragma unroll
                for (int i = 0; i < W; ++i) s += Wl[i * W + j] * gz[i];
                ga[j] = s;
            }
        }
    }
    // dL/da_0 and the table contributions, level by level
    const float *W1 = h.theta + h.loff[1];
    constexpr int nv = 1 << DIM;
    for (int l = 0; l < h.levels; ++l) {
        float d0 = 0.f, d1 = 0.f;
#pragma unroll
        for (int i = 0; i < W; ++i) {
            d0 += W1[(size_t)i * K + 2 * l] * gz[i];
            d1 += W1[(size_t)i * K + 2 * l + 1] * gz[i];
        }
        unsigned vid[8];
        float vw[8];
        (void)hash_level<DIM>(h, l, ix, iy, iz, vid, vw);
        const size_t base = ((size_t)t * h.levels + l) * nv;
#pragma unroll
        for (int m = 0; m < nv; ++m) {
            ckey[base + m] = (uint32_t)l * (uint32_t)h.T + vid[m];
            cpos[base + m] = (uint32_t)(base + m);
            cval[base + m] = make_float2(vw[m] * d0, vw[m] * d1);
        }
    }
}

// dW partial sums: entry e of the MLP (layer-major, W then b per layer),
// over points [s * S, min(k, (s + 1) * S)) in order.
__global__ __launch_bounds__(256) void k_hash_dw(HashDev h, const float *__restrict__ rows,
                                                 int R, long long k, int S, long long n_mlp,
                                                 float *__restrict__ part) {
    const long long e = (long long)blockIdx.x * 256 + threadIdx.x;
    const int s = blockIdx.y;
    if (e >= n_mlp) return;
    // locate the layer
    int l = 1;
    while (l <= h.L && e >= h.loff[l + 1] - h.loff[1]) ++l;
    const long long le = e - (h.loff[l] - h.loff[1]);
    const int fi = l == 1 ? h.K : h.W;
    const int fo = l == h.L + 1 ? 1 : h.W;
    const int dof = l == h.L + 1 ? h.K + 2 * h.L * h.W : h.K + h.L * h.W + (l - 1) * h.W;
    const int aof = l == 1 ? 0 : h.K + (l - 2) * h.W;
    int i, j;
    if (le < (long long)fo * fi) {
        i = (int)(le / fi);
        j = (int)(le % fi);
    } else {
        i = (int)(le - (long long)fo * fi);
        j = -1;  // bias
    }
    const long long p0 = (long long)s * S, p1 = min(k, p0 + S);
    // four interleaved partial sums (points p0 + 4q + r go to sum r), added
    // in a fixed order at the end
    float acc[4] = {0.f, 0.f, 0.f, 0.f};
    const float *dp = rows + (size_t)p0 * R + dof + i;
    const float *ap = rows + (size_t)p0 * R + (j >= 0 ? aof + j : 0);
    long long p = p0;
    for (; p + 4 <= p1; p += 4, dp += 4 * (size_t)R, ap += 4 * (size_t)R) {
#pragma unroll
        for (int r = 0; r < 4; ++r) {
            const float dv = dp[(size_t)r * R];
            acc[r] += j >= 0 ? dv * ap[(size_t)r * R] : dv;
        }
    }
    for (int r = 0; p < p1; ++p, ++r, dp += R, ap += R) acc[r] += j >= 0 ? dp[0] * ap[0] : dp[0];
    part[(size_t)s * n_mlp + e] = (acc[0] + acc[1]) + (acc[2] + acc[3]);
}

__global__ __launch_bounds__(256) void k_hash_dw_sum(const float *__restrict__ part, int ns,
                                                     long long n_mlp, long long off,
                                                     float *__restrict__ grad) {
    const long long e = (long long)blockIdx.x * 256 + threadIdx.x;
    if (e >= n_mlp) return;
    float s = 0.f;
    for (int q = 0; q < ns; ++q) s += part[(size_t)q * n_mlp + e];
    grad[off + e] = s;
}

__global__ __launch_bounds__(256) void k_hash_zero(float *__restrict__ p, long long n) {
    const long long i = (long long)blockIdx.x * 256 + threadIdx.x;
    if (i < n) p[i] = 0.f;
}

// Table gradient: one thread per run of equal sorted keys sums the run in
// sorted (= contribution) order.
__global__ __launch_bounds__(256) void k_hash_runs(const uint32_t *__restrict__ key,
                                                   const uint32_t *__restrict__ pos,
                                                   const float2 *__restrict__ val, long long n,
                                                   float *__restrict__ grad) {
    const long long s = (long long)blockIdx.x * 256 + threadIdx.x;
    if (s >= n) return;
    const uint32_t kk = key[s];
    if (s > 0 && key[s - 1] == kk) return;
    // eight sorted entries per iteration, their loads issued together; keys
    // are ascending, so the run ends at the first different key
    float gx = 0.f, gy = 0.f;
    for (long long q = s; q < n; q += 8) {
        uint32_t kq[8], pq[8];
        float2 vq[8];
#pragma unroll
        for (int i = 0; i < 8; ++i) kq[i] = q + i < n ? key[q + i] : kk + 1u;
#pragma unroll
        for (int i = 0; i < 8; ++i) pq[i] = kq[i] == kk ? pos[q + i] : 0u;
#pragma unroll
        for (int i = 0; i < 8; ++i) vq[i] = kq[i] == kk ? val[pq[i]] : make_float2(0.f, 0.f);
#pragma unroll
        for (int i = 0; i < 8; ++i)
            if (kq[i] == kk) {
                gx += vq[i].x;
                gy += vq[i].y;
            }
        if (kq[7] != kk) break;
    }
    grad[2 * (size_t)kk] = gx;
    grad[2 * (size_t)kk + 1] = gy;
}

// --------------------------------------------------------------- host side
static HashDev hash_dev(const inrct_model *m, const float *theta) {
    HashDev h{};
    h.theta = theta;
    h.fov = m->fov.dev(m->dim);
    h.N = m->N;
    h.dim = m->dim;
    h.levels = m->arch.hash_levels;
    h.T = 1 << m->arch.hash_log2_size;
    h.W = m->arch.width;
    h.L = m->arch.depth;
    h.K = 2 * h.levels;
    for (int l = 0; l < h.levels; ++l) {
        h.res[l] = m->hash_res[l];
        long long v = 1;
        for (int i = 0; i < m->dim; ++i) v *= (long long)m->hash_res[l] + 1;
        h.dense[l] = v <= h.T ? 1 : 0;
    }
    for (int l = 1; l <= h.L + 1; ++l) h.loff[l] = m->loff[l];
    return h;
}

#define HASH_DISPATCH_D(W_, D_, FN, ...)                                            \
    do {                                                                            \
        if ((W_) == 16) FN<16, 4, D_>(__VA_ARGS__);                                 \
        else if ((W_) == 32) FN<32, 4, D_>(__VA_ARGS__);                            \
        else FN<64, 2, D_>(__VA_ARGS__);                                            \
    } while (0)
#define HASH_DISPATCH(W_, DIM_, FN, ...)                                             \
    do {                                                                            \
        if ((DIM_) == 3) HASH_DISPATCH_D(W_, 3, FN, __VA_ARGS__);                   \
        else HASH_DISPATCH_D(W_, 2, FN, __VA_ARGS__);                               \
    } while (0)

template <int W, int LM, int DIM>
static void launch_hash_eval(const HashDev &h, long long n, int mode, const int32_t *idx,
                             float *out, hipStream_t s) {
    hipLaunchKernelGGL((k_hash_eval<W, LM, DIM>), dim3((unsigned)cdiv(n, 256)), dim3(256), 0, s, h,
                       n, mode, idx, out);
}

void hash_eval(inrct_model *m, const float *theta, const int32_t *idx, long long n,
               float *out, hipStream_t s) {
    if (n <= 0) return;
    const HashDev h = hash_dev(m, theta);
    HASH_DISPATCH(h.W, h.dim, launch_hash_eval, h, n, idx ? 1 : 0, idx, out, s);
    INRCT_CHECK_LAUNCH();
}

template <int W, int LM, int DIM>
static void launch_hash_vjp(const HashDev &h, const int32_t *idx, long long k, const float *v,
                            int v_compact, float scale, float *rows, int R, uint32_t *ckey,
                            uint32_t *cpos, float2 *cval, hipStream_t s) {
    hipLaunchKernelGGL((k_hash_vjp<W, LM, DIM>), dim3((unsigned)cdiv(k, 256)), dim3(256), 0, s, h,
                       idx, k, v, v_compact, scale, rows, R, ckey, cpos, cval);
}

void hash_vjp(inrct_model *m, const float *theta, const int32_t *idx, long long k,
              const float *v, int v_compact, double scale, float *grad, hipStream_t s) {
    const HashDev h = hash_dev(m, theta);
    const long long n_tab = (long long)h.levels * h.T * 2;
    const long long n_mlp = m->n_params - n_tab;
    hipLaunchKernelGGL(k_hash_zero, dim3((unsigned)cdiv(n_tab, 256)), dim3(256), 0, s, grad,
                       n_tab);
    INRCT_CHECK_LAUNCH();
    if (k <= 0) {
        hipLaunchKernelGGL(k_hash_zero, dim3((unsigned)cdiv(n_mlp, 256)), dim3(256), 0, s,
                           grad + n_tab, n_mlp);
        INRCT_CHECK_LAUNCH();
        return;
    }
    const int R = m->hash_row;
    const int nv = m->dim == 3 ? 8 : 4;
    const long long nc = k * h.levels * nv;
    uint32_t *ckey = m->hash_key.as<uint32_t>(), *cpos = m->hash_pos.as<uint32_t>();
    uint32_t *skey = m->hash_skey.as<uint32_t>(), *spos = m->hash_spos.as<uint32_t>();
    float2 *cval = m->hash_val.as<float2>();
    float *rows = m->hash_rows.as<float>();
    HASH_DISPATCH(h.W, h.dim, launch_hash_vjp, h, idx, k, v, v_compact, (float)scale, rows, R,
                  ckey, cpos, cval, s);
    INRCT_CHECK_LAUNCH();
    // MLP weight gradients: slices of kHashSlice points, then their sum
    const int ns = (int)cdiv(k, kHashSlice);
    hipLaunchKernelGGL(k_hash_dw, dim3((unsigned)cdiv(n_mlp, 256), (unsigned)ns), dim3(256), 0,
                       s, h, rows, R, k, kHashSlice, n_mlp, m->hash_part.as<float>());
    INRCT_CHECK_LAUNCH();
    hipLaunchKernelGGL(k_hash_dw_sum, dim3((unsigned)cdiv(n_mlp, 256)), dim3(256), 0, s,
                       m->hash_part.as<float>(), ns, n_mlp, n_tab, grad);
    INRCT_CHECK_LAUNCH();
    // table gradients: stable sort of the contributions by entry, run sums
    size_t tb = m->hash_tmp.bytes;
    INRCT_CHECK_HIP(hipcub::DeviceRadixSort::SortPairs(m->hash_tmp.ptr, tb, ckey, skey, cpos,
                                                       spos, (int)nc, 0, m->hash_key_bits, s));
    hipLaunchKernelGGL(k_hash_runs, dim3((unsigned)cdiv(nc, 256)), dim3(256), 0, s, skey, spos,
                       cval, nc, grad);
    INRCT_CHECK_LAUNCH();
}

void hash_setup(inrct_model *m, Arena &ar) {
    const inr_arch &a = m->arch;
    const int Lh = a.hash_levels;
    const double b = Lh == 1 ? 1.0
                             : exp((log((double)a.hash_max_res) - log((double)a.hash_base_res)) /
                                   (double)(Lh - 1));
    for (int l = 0; l < Lh; ++l)
        m->hash_res[l] = (int)floor((double)a.hash_base_res * pow(b, (double)l) + 1e-6);
    const long long T = 1LL << a.hash_log2_size;
    const int K = 2 * Lh, W = a.width, L = a.depth;
    m->loff.assign(L + 2, 0);
    long long off = (long long)Lh * T * 2;
    for (int l = 1; l <= L + 1; ++l) {
        m->loff[l] = off;
        const int fi = l == 1 ? K : W, fo = l == L + 1 ? 1 : W;
        off += (long long)fi * fo + fo;
    }
    m->n_params = off;
    upload(ar, m->d_loff, m->loff);
    const long long kmax = m->max_k;
    m->hash_row = K + 2 * L * W + 1;
    m->hash_rows.alloc(ar, sizeof(float) * (size_t)kmax * m->hash_row);
    const int nv = m->dim == 3 ? 8 : 4;
    const long long nc = kmax * Lh * nv;
    INRCT_REQUIRE(nc < (1LL << 31), "too many hash-table contributions (max_k x levels x 2^d)");
    m->hash_key.alloc(ar, sizeof(uint32_t) * nc);
    m->hash_pos.alloc(ar, sizeof(uint32_t) * nc);
    m->hash_skey.alloc(ar, sizeof(uint32_t) * nc);
    m->hash_spos.alloc(ar, sizeof(uint32_t) * nc);
    m->hash_val.alloc(ar, sizeof(float2) * nc);
    int bits = 1;
    while ((1LL << bits) < (long long)Lh * T) ++bits;
    m->hash_key_bits = bits;
    size_t tb = 0;
    INRCT_CHECK_HIP(hipcub::DeviceRadixSort::SortPairs(nullptr, tb, (uint32_t *)nullptr,
                                                       (uint32_t *)nullptr, (uint32_t *)nullptr,
                                                       (uint32_t *)nullptr, (int)nc, 0, bits));
    m->hash_tmp.alloc(ar, std::max<size_t>(tb, 256));
    const long long n_mlp = m->n_params - (long long)Lh * T * 2;
    m->hash_part.alloc(ar, sizeof(float) * (size_t)cdiv(kmax, kHashSlice) * n_mlp);
}

}  // namespace inrct
