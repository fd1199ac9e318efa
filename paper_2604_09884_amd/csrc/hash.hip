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
// stable LSD radix sort (equal entries keep the points' order; below) and
// each entry's run is summed in order.  No atomics: results are bitwise
// repeatable.
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

// f_theta at one grid point, for E: hash_forward's arithmetic in its order,
// with the last hidden layer fused with the output (each unit's activation
// goes into f as soon as it is formed, in unit order) and that layer's unit
// loop kept rolled, so only one layer of activations is held in registers.
template <int W, int LMAX, int DIM>
__device__ __forceinline__ float hash_eval_point(const HashDev &h, int ix, int iy, int iz) {
    const float *W1 = h.theta + h.loff[1];
    float a[W];
    {
        float z[W];
#pragma unroll
        for (int i = 0; i < W; ++i) z[i] = W1[(size_t)W * h.K + i];
        for (int l = 0; l < h.levels; ++l) {
            const float2 e = hash_level<DIM>(h, l, ix, iy, iz, nullptr, nullptr);
#pragma unroll
            for (int i = 0; i < W; ++i)
                z[i] += W1[(size_t)i * h.K + 2 * l] * e.x + W1[(size_t)i * h.K + 2 * l + 1] * e.y;
        }
#pragma unroll
        for (int i = 0; i < W; ++i) a[i] = fmaxf(z[i], 0.f);
    }
    const float *Wo = h.theta + h.loff[h.L + 1];
    float f = Wo[W];
    if (h.L == 1) {
#pragma unroll
        for (int j = 0; j < W; ++j) f += Wo[j] * a[j];
        return f;
    }
#pragma unroll
    for (int l = 1; l < LMAX; ++l) {
        const float *Wl = h.theta + h.loff[l + 1];
        if (l == h.L - 1) {
#pragma unroll 1
            for (int i = 0; i < W; ++i) {
                float s = Wl[W * W + i];
#pragma unroll
                for (int j = 0; j < W; ++j) s += Wl[i * W + j] * a[j];
                f += Wo[i] * fmaxf(s, 0.f);
            }
            break;
        }
        float b[W];
#pragma unroll
        for (int i = 0; i < W; ++i) {
            float s = Wl[W * W + i];
#pragma unroll
            for (int j = 0; j < W; ++j) s += Wl[i * W + j] * a[j];
            b[i] = fmaxf(s, 0.f);
        }
#pragma unroll
        for (int i = 0; i < W; ++i) a[i] = b[i];
    }
    return f;
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
    out[mode == 0 ? g : q] = hash_eval_point<W, LMAX, DIM>(h, ix, iy, iz);
}

// Row of point t (R floats): a_0 (K) | a_1..a_L (W each) | d_1..d_L (W each)
// | d_out.  Contributions of point t: (level, vertex) keys and the two
// weighted feature gradients.
template <int W, int LMAX, int DIM>
__global__ __launch_bounds__(64) void k_hash_vjp(HashDev h, const int32_t *__restrict__ idx,
                                                  long long k, const float *__restrict__ v,
                                                  int v_compact, float scale,
                                                  float *__restrict__ rows, int R,
                                                  uint32_t *__restrict__ ckey,
                                                  uint32_t *__restrict__ cpos,
                                                  float2 *__restrict__ cval) {
    const long long t = (long long)blockIdx.x * 64 + threadIdx.x;
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

// ------------------------------------------------ stable LSD radix sort
// Sorts (key, position) pairs by the low `bits` bits of the key, eight bits
// per pass; the last pass moves the contribution values themselves (gathered
// through the positions), so the run sums below read them contiguously.
// Items are taken in tiles of kRsTile in index order; within a tile, item
// it * 256 + thread comes before item (it + 1) * 256 + thread, and within a
// round of 256 the wave and lane order is the index order.  An item's place
// is its digit's start in the output, plus the items of that digit in earlier
// tiles, earlier rounds, earlier waves of its round and lower lanes of its
// wave (found with ballots), so equal keys keep their input order.  Counts
// are per wave and per digit in LDS: no atomics.
constexpr int kRsItems = 8, kRsTile = 256 * kRsItems, kRsDigits = 256;

// lanes of this wave (among `live`) whose digit equals this lane's
__device__ __forceinline__ uint64_t rs_peers(unsigned dg, uint64_t live) {
    uint64_t m = live;
#pragma unroll
    for (int b = 0; b < 8; ++b) {
        const uint64_t on = __ballot((dg >> b) & 1u);
        m &= ((dg >> b) & 1u) ? on : ~on;
    }
    return m;
}

// number of lanes below this one set in m
__device__ __forceinline__ int rs_below(uint64_t m) {
    return (int)__builtin_amdgcn_mbcnt_hi((unsigned)(m >> 32),
                                          __builtin_amdgcn_mbcnt_lo((unsigned)m, 0u));
}

// inclusive scan over the 256 threads of the block; *total = the block's sum
__device__ __forceinline__ uint32_t rs_block_scan(uint32_t x, uint32_t *sw, uint32_t *total) {
    const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
#pragma unroll
    for (int d = 1; d < 64; d <<= 1) {
        const uint32_t y = __shfl_up(x, d);
        if (lane >= d) x += y;
    }
    if (lane == 63) sw[w] = x;
    __syncthreads();
    uint32_t off = 0, tot = 0;
#pragma unroll
    for (int q = 0; q < 4; ++q) {
        const uint32_t v = sw[q];
        off += q < w ? v : 0u;
        tot += v;
    }
    __syncthreads();
    *total = tot;
    return x + off;
}

// per tile and digit: the number of items (cnt[digit * ntiles + tile])
__global__ __launch_bounds__(256) void k_rs_count(const uint32_t *__restrict__ key, long long n,
                                                  int sh, int ntiles, uint32_t *__restrict__ cnt) {
    __shared__ uint32_t wc[4][kRsDigits];
    const int tid = threadIdx.x, w = tid >> 6;
#pragma unroll
    for (int q = 0; q < 4; ++q) wc[q][tid] = 0u;
    const long long base = (long long)blockIdx.x * kRsTile;
    uint32_t kk[kRsItems];
#pragma unroll
    for (int it = 0; it < kRsItems; ++it) {
        const long long i = base + it * 256 + tid;
        kk[it] = i < n ? key[i] : 0u;
    }
    __syncthreads();
#pragma unroll
    for (int it = 0; it < kRsItems; ++it) {
        const bool ok = base + it * 256 + tid < n;
        const unsigned dg = (kk[it] >> sh) & 255u;
        const uint64_t pm = rs_peers(dg, __ballot(ok));
        // one lane per digit group (its lowest) adds the group's size; the
        // wave's LDS accesses are carried out in order
        if (ok && rs_below(pm) == 0) wc[w][dg] += (uint32_t)__popcll(pm);
    }
    __syncthreads();
    cnt[(size_t)tid * ntiles + blockIdx.x] = wc[0][tid] + wc[1][tid] + wc[2][tid] + wc[3][tid];
}

// one block per digit: exclusive prefix of the digit's tile counts, in place;
// tot[digit] = the digit's total
__global__ __launch_bounds__(256) void k_rs_scan(uint32_t *__restrict__ cnt, int ntiles,
                                                 uint32_t *__restrict__ tot) {
    __shared__ uint32_t sw[4];
    uint32_t *c = cnt + (size_t)blockIdx.x * ntiles;
    uint32_t carry = 0;
    for (int b0 = 0; b0 < ntiles; b0 += 256) {
        const int b = b0 + threadIdx.x;
        const uint32_t x = b < ntiles ? c[b] : 0u;
        uint32_t t;
        const uint32_t inc = rs_block_scan(x, sw, &t);
        if (b < ntiles) c[b] = carry + inc - x;
        carry += t;
    }
    if (threadIdx.x == 0) tot[blockIdx.x] = carry;
}

// stable scatter of one tile; LAST moves val[pos] instead of pos
template <bool LAST>
__global__ __launch_bounds__(256) void k_rs_scatter(
    const uint32_t *__restrict__ key, const uint32_t *__restrict__ pos, long long n, int sh,
    int ntiles, const uint32_t *__restrict__ cnt, const uint32_t *__restrict__ tot,
    uint32_t *__restrict__ key_out, uint32_t *__restrict__ pos_out,
    const float2 *__restrict__ val, float2 *__restrict__ val_out) {
    __shared__ uint32_t run[kRsDigits], wc[4][kRsDigits], sw[4];
    const int tid = threadIdx.x, w = tid >> 6;
    const long long base = (long long)blockIdx.x * kRsTile;
    uint32_t kk[kRsItems], pp[kRsItems];
#pragma unroll
    for (int it = 0; it < kRsItems; ++it) {
        const long long i = base + it * 256 + tid;
        kk[it] = i < n ? key[i] : 0u;
        pp[it] = i < n ? pos[i] : 0u;
    }
    // run[d]: where this tile's next item of digit d goes
    const uint32_t td = tot[tid];
    uint32_t all;
    const uint32_t inc = rs_block_scan(td, sw, &all);
    run[tid] = inc - td + cnt[(size_t)tid * ntiles + blockIdx.x];
#pragma unroll
    for (int q = 0; q < 4; ++q) wc[q][tid] = 0u;
    __syncthreads();
#pragma unroll
    for (int it = 0; it < kRsItems; ++it) {
        const bool ok = base + it * 256 + tid < n;
        const unsigned dg = (kk[it] >> sh) & 255u;
        const uint64_t pm = rs_peers(dg, __ballot(ok));
        const int r = rs_below(pm);
        if (ok && r == 0) wc[w][dg] = (uint32_t)__popcll(pm);
        __syncthreads();
        if (ok) {
            uint32_t o = run[dg] + (uint32_t)r;
            for (int q = 0; q < w; ++q) o += wc[q][dg];
            key_out[o] = kk[it];
            if (LAST) val_out[o] = val[pp[it]];
            else pos_out[o] = pp[it];
        }
        __syncthreads();
        run[tid] += wc[0][tid] + wc[1][tid] + wc[2][tid] + wc[3][tid];
#pragma unroll
        for (int q = 0; q < 4; ++q) wc[q][tid] = 0u;
        __syncthreads();
    }
}

// Table gradient: one thread per run of equal sorted keys sums the run in
// sorted (= contribution) order.
__global__ __launch_bounds__(256) void k_hash_runs(const uint32_t *__restrict__ key,
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
        uint32_t kq[8];
        float2 vq[8];
#pragma unroll
        for (int i = 0; i < 8; ++i) kq[i] = q + i < n ? key[q + i] : kk + 1u;
#pragma unroll
        for (int i = 0; i < 8; ++i) vq[i] = kq[i] == kk ? val[q + i] : make_float2(0.f, 0.f);
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
    hipLaunchKernelGGL((k_hash_vjp<W, LM, DIM>), dim3((unsigned)cdiv(k, 64)), dim3(64), 0, s, h,
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
    // table gradients: stable sort of the contributions by entry (eight key
    // bits a pass, ping-ponging between the two key / position buffers), run
    // sums
    const int ntiles = (int)cdiv(nc, kRsTile);
    const int passes = (int)cdiv(m->hash_key_bits, 8);
    uint32_t *cnt = m->hash_cnt.as<uint32_t>(), *tot = cnt + (size_t)kRsDigits * ntiles;
    float2 *sval = m->hash_sval.as<float2>();
    uint32_t *kin = ckey, *pin = cpos, *kout = skey, *pout = spos;
    for (int p = 0; p < passes; ++p) {
        const int sh = 8 * p;
        hipLaunchKernelGGL(k_rs_count, dim3((unsigned)ntiles), dim3(256), 0, s, kin, nc, sh,
                           ntiles, cnt);
        INRCT_CHECK_LAUNCH();
        hipLaunchKernelGGL(k_rs_scan, dim3((unsigned)kRsDigits), dim3(256), 0, s, cnt, ntiles,
                           tot);
        INRCT_CHECK_LAUNCH();
        if (p + 1 < passes)
            hipLaunchKernelGGL(k_rs_scatter<false>, dim3((unsigned)ntiles), dim3(256), 0, s, kin,
                               pin, nc, sh, ntiles, cnt, tot, kout, pout, cval, sval);
        else
            hipLaunchKernelGGL(k_rs_scatter<true>, dim3((unsigned)ntiles), dim3(256), 0, s, kin,
                               pin, nc, sh, ntiles, cnt, tot, kout, pout, cval, sval);
        INRCT_CHECK_LAUNCH();
        std::swap(kin, kout);
        std::swap(pin, pout);
    }
    hipLaunchKernelGGL(k_hash_runs, dim3((unsigned)cdiv(nc, 256)), dim3(256), 0, s, kin, sval,
                       nc, grad);
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
    m->hash_sval.alloc(ar, sizeof(float2) * nc);
    int bits = 1;
    while ((1LL << bits) < (long long)Lh * T) ++bits;
    m->hash_key_bits = bits;
    m->hash_cnt.alloc(ar, sizeof(uint32_t) * ((size_t)kRsDigits * cdiv(nc, kRsTile) + kRsDigits));
    const long long n_mlp = m->n_params - (long long)Lh * T * 2;
    m->hash_part.alloc(ar, sizeof(float) * (size_t)cdiv(kmax, kHashSlice) * n_mlp);
}

}  // namespace inrct
