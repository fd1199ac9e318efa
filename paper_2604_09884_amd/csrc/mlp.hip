// INR f_theta on matrix cores: grid evaluation E (Sec. III), point
// evaluation, and the subsampled Jacobian-transpose product of Eq. (2).
//
// Layout of the forward GEMMs.  Every hidden layer is Y^T = W A^T with the
// output features as the MFMA M dimension (32-row tiles), the layer inputs
// as K and 32 points as N.  A 32x32 MFMA result leaves, in lane l, point
// l % 32 and rows 8*(r/4) + 4*(l/32) + r%4 (r = 0..15) of the tile.  Those
// are exactly the K values lane l must supply as the next layer's B
// operand if the next layer's K order is permuted accordingly, so
// activations stay in registers from layer to layer and only the packed
// weights (A operands, permuted on the device by k_pack) are read from
// memory.  The bias is one extra K step whose B operand is the constant 1.
//
// Two precisions: BF16 operands with FP32 accumulation
// (v_mfma_f32_32x32x16_bf16, 16 K per step) and FP32
// (v_mfma_f32_32x32x2f32, 2 K per step).
//
// The VJP recomputes the forward pass per 32-point tile, stores the tile's
// activations and back-propagated deltas for one bounded chunk of points,
// then forms dW = delta A^T for every layer with a split-K MFMA GEMM over the
// chunk's points.  Split-K partials accumulate across chunks in a fixed
// order and are summed in a fixed order at the end: no atomics.
#include <math.h>

#include "model.h"

namespace inrct {

typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));
typedef float f32x16 __attribute__((ext_vector_type(16)));

static const int kMaxDepth = 8;

struct MlpDev {
    int kind;        // INRCT_FFN / INRCT_SIREN
    int d, F, W, L;  // input dim, frequencies, width, hidden layers
    float omega0;
    const void *frag;    // forward A fragments (layers 1..L for FFN, 2..L SIREN)
    const void *fragT;   // transposed fragments for deltas (layers 2..L)
    const float *w_out;  // [W]
    const float *b_out;  // [1]
    const float *W1;     // SIREN layer 1 [W][d]
    const float *b1;     // SIREN layer 1 [W]
    const float *B;      // FFN Fourier matrix [F][d]
    long long off[kMaxDepth + 2];   // fragment offset of layer l (1-based)
    long long offT[kMaxDepth + 2];
    const float *theta;             // parameters (for the biases)
    long long boff[kMaxDepth + 2];  // theta offset of the bias of layer l (1-based)
    FovDev fov;
};

template <bool BF>
struct Prec;

template <>
struct Prec<true> {
    typedef bf16x8 Op;
    static constexpr int KPS = 16;
    typedef __bf16 Store;
    static __device__ __forceinline__ f32x16 mma(Op a, Op b, f32x16 c) {
        return __builtin_amdgcn_mfma_f32_32x32x16_bf16(a, b, c, 0, 0, 0);
    }
};

template <>
struct Prec<false> {
    typedef float Op;
    static constexpr int KPS = 2;
    typedef float Store;
    static __device__ __forceinline__ f32x16 mma(Op a, Op b, f32x16 c) {
        return __builtin_amdgcn_mfma_f32_32x32x2f32(a, b, c, 0, 0, 0);
    }
};

// K steps of layer l (including the bias step) and of the transposed pass.
__host__ __device__ inline int layer_K(int kind, int F, int d, int W, int l) {
    return l == 1 ? (kind == INRCT_FFN ? 2 * F : d) : W;
}
__host__ __device__ inline int ksteps(int K, int kps) { return K / kps + 1; }

// Row of the 32-row tile held by lane-half h in accumulator slot r.
__host__ __device__ inline int crow(int r, int h) { return 8 * (r / 4) + 4 * h + (r % 4); }

// Input feature of layer l >= 2 supplied at k-step s, lane-half h, slot p.
__host__ __device__ inline int chain_feature(bool bf, int s, int h, int p) {
    if (bf) {
        const int r = 8 * (s % 2) + p;
        return 32 * (s / 2) + crow(r, h);
    }
    const int r = s % 16;
    return 32 * (s / 16) + crow(r, h);
}

// Encoding feature (column of W_1) at k-step s, lane-half h, slot p (FFN).
__host__ __device__ inline int enc_feature(bool bf, int F, int s, int h, int p) {
    if (bf) {
        const int f = 8 * s + 4 * h + p / 2;
        return (p % 2) == 0 ? f : F + f;
    }
    return h == 0 ? s : F + s;
}

// ------------------------------------------------------------ weight pack
// One thread per (fragment, lane, slot).  theta layout: per layer W then b.
__global__ void k_pack(MlpDev m, const float *__restrict__ theta, int bf, void *frag,
                       void *fragT, long long nfrag, long long nfragT,
                       const long long *__restrict__ loff,
                       const int *__restrict__ flayer, const int *__restrict__ fmt,
                       const int *__restrict__ fs) {
    const int slots = bf ? 8 : 1;
    const long long total = (nfrag + nfragT) * 64 * slots;
    const long long t = (long long)blockIdx.x * 256 + threadIdx.x;
    if (t >= total) return;
    const int p = (int)(t % slots);
    const int lane = (int)((t / slots) % 64);
    const long long fi = t / (slots * 64);
    const bool trans = fi >= nfrag;
    const int l = flayer[fi], mt = fmt[fi], s = fs[fi];
    const int i = lane % 32, h = lane / 32;
    const int W = m.W;
    const int K = layer_K(m.kind, m.F, m.d, W, l);
    const float *Wl = theta + loff[l];
    const float *bl = Wl + (long long)K * W;
    float val = 0.f;
    if (!trans) {
        const int o = 32 * mt + i;
        const int KS = ksteps(K, bf ? 16 : 2);
        if (s >= KS) {
            val = 0.f;  // padding k-step
        } else if (s == KS - 1) {
            val = (h == 0 && p == 0) ? bl[o] : 0.f;
        } else {
            const int col = (l == 1) ? enc_feature(bf, m.F, s, h, p) : chain_feature(bf, s, h, p);
            val = Wl[(long long)o * K + col];
        }
    } else {
        const int o = chain_feature(bf, s, h, p);  // output feature of layer l
        val = Wl[(long long)o * K + 32 * mt + i];
    }
    const long long idx = (trans ? (fi - nfrag) : fi) * 64 + lane;
    if (bf) {
        __bf16 *dst = (__bf16 *)(trans ? fragT : frag);
        dst[idx * 8 + p] = (__bf16)val;
    } else {
        float *dst = (float *)(trans ? fragT : frag);
        dst[idx] = val;
    }
}

// ---------------------------------------------------------- forward core
template <int ACT>
__device__ __forceinline__ float act_fn(float z, float w0) {
    if constexpr (ACT == INRCT_FFN) return fmaxf(z, 0.f);
    else return sinf(w0 * z);
}
template <int ACT>
__device__ __forceinline__ float act_grad(float z, float w0) {
    if constexpr (ACT == INRCT_FFN) return z > 0.f ? 1.f : 0.f;
    else return w0 * cosf(w0 * z);
}

// sin and cos of 2 pi t (t in turns), reduced to [-1/2, 1/2] first.
__device__ __forceinline__ void sincos_turns(float t, float *s, float *c) {
    const float r = t - rintf(t);
    *s = sinpif(2.f * r);
    *c = cospif(2.f * r);
}

// Sink for activations / pre-activation derivatives during the VJP.
template <bool BF>
struct ActSink {
    typename Prec<BF>::Store *act;  // base of activation scratch
    float *sig;                     // SIREN derivative scratch (or null)
    long long P;                    // points per chunk (row stride)
    long long act_off[kMaxDepth + 2];
    long long sig_off[kMaxDepth + 2];
    uint4 *mask;                    // ReLU masks: [layer-1][P/32 tiles][64 lanes]
};

// 128 bits of "z > 0" for accumulator slots i = 16 mt + r (lane's point).
template <int MT>
__device__ __forceinline__ uint4 relu_bits(const f32x16 (&acc)[MT]) {
    unsigned w[4] = {0u, 0u, 0u, 0u};
#pragma unroll
    for (int mt = 0; mt < MT; ++mt)
#pragma unroll
        for (int r = 0; r < 16; ++r) {
            const int i = 16 * mt + r;
            w[i >> 5] |= (acc[mt][r] > 0.f ? 1u : 0u) << (i & 31);
        }
    return make_uint4(w[0], w[1], w[2], w[3]);
}

__device__ __forceinline__ float mask_bit(const uint4 &b, int i) {
    const unsigned w = i < 32 ? b.x : (i < 64 ? b.y : (i < 96 ? b.z : b.w));
    return (w >> (i & 31)) & 1u ? 1.f : 0.f;
}

template <int W, int NT, bool BF, int ACT, bool STORE>
__device__ __forceinline__ void mlp_forward(const MlpDev &m, const float (&xc)[NT][3],
                                            f32x16 (&acc)[NT][W / 32],
                                            const ActSink<BF> &sink,
                                            const int (&pcol)[NT]) {
    typedef Prec<BF> PR;
    typedef typename PR::Op Op;
    constexpr int MT = W / 32;
    constexpr int KPS = PR::KPS;
    const int lane = threadIdx.x & 63;
    const int h = lane >> 5;
    const int L = m.L;
    const Op *frag = (const Op *)m.frag;

    Op one_b;
    if constexpr (BF) {
        for (int p = 0; p < 8; ++p) one_b[p] = (__bf16)((h == 0 && p == 0) ? 1.f : 0.f);
    } else {
        one_b = h == 0 ? 1.f : 0.f;
    }

#pragma unroll
    for (int nt = 0; nt < NT; ++nt)
#pragma unroll
        for (int mt = 0; mt < MT; ++mt) acc[nt][mt] = (f32x16){0};

    // ---------------- layer 1
    if constexpr (ACT == INRCT_FFN) {
        const int F = m.F;
        const int KS = ksteps(2 * F, KPS);
        const Op *fr = frag + m.off[1] * 64;
        for (int s = 0; s < KS - 1; ++s) {
            Op bop[NT];
            if constexpr (BF) {
#pragma unroll
                for (int q = 0; q < 4; ++q) {
                    const int f = 8 * s + 4 * h + q;
                    const float bx = m.B[f * m.d], by = m.B[f * m.d + 1];
                    const float bz = m.d == 3 ? m.B[f * m.d + 2] : 0.f;
#pragma unroll
                    for (int nt = 0; nt < NT; ++nt) {
                        const float t = fmaf(bz, xc[nt][2], fmaf(by, xc[nt][1], bx * xc[nt][0]));
                        float sn, cs;
                        sincos_turns(t, &sn, &cs);
                        bop[nt][2 * q] = (__bf16)sn;
                        bop[nt][2 * q + 1] = (__bf16)cs;
                        if constexpr (STORE) {
                            if (pcol[nt] >= 0) {
                                sink.act[sink.act_off[0] + (long long)f * sink.P + pcol[nt]] = (__bf16)sn;
                                sink.act[sink.act_off[0] + (long long)(F + f) * sink.P + pcol[nt]] = (__bf16)cs;
                            }
                        }
                    }
                }
            } else {
                const int f = s;
                const float bx = m.B[f * m.d], by = m.B[f * m.d + 1];
                const float bz = m.d == 3 ? m.B[f * m.d + 2] : 0.f;
#pragma unroll
                for (int nt = 0; nt < NT; ++nt) {
                    const float t = fmaf(bz, xc[nt][2], fmaf(by, xc[nt][1], bx * xc[nt][0]));
                    float sn, cs;
                    sincos_turns(t, &sn, &cs);
                    bop[nt] = h == 0 ? sn : cs;
                    if constexpr (STORE) {
                        if (pcol[nt] >= 0)
                            sink.act[sink.act_off[0] + (long long)(h == 0 ? f : F + f) * sink.P + pcol[nt]] = bop[nt];
                    }
                }
            }
#pragma unroll
            for (int mt = 0; mt < MT; ++mt) {
                const Op a = fr[((long long)s * MT + mt) * 64 + lane];
#pragma unroll
                for (int nt = 0; nt < NT; ++nt) acc[nt][mt] = PR::mma(a, bop[nt], acc[nt][mt]);
            }
        }
#pragma unroll
        for (int mt = 0; mt < MT; ++mt) {
            const Op a = fr[((long long)(KS - 1) * MT + mt) * 64 + lane];
#pragma unroll
            for (int nt = 0; nt < NT; ++nt) acc[nt][mt] = PR::mma(a, one_b, acc[nt][mt]);
        }
    } else {
        // SIREN layer 1 on the vector units: z = W1 x + b1 in C layout
#pragma unroll
        for (int mt = 0; mt < MT; ++mt)
#pragma unroll
            for (int r = 0; r < 16; ++r) {
                const int o = 32 * mt + crow(r, h);
                const float w0 = m.W1[o * m.d], w1 = m.W1[o * m.d + 1];
                const float w2 = m.d == 3 ? m.W1[o * m.d + 2] : 0.f;
                const float bb = m.b1[o];
#pragma unroll
                for (int nt = 0; nt < NT; ++nt)
                    acc[nt][mt][r] = fmaf(w2, xc[nt][2], fmaf(w1, xc[nt][1], fmaf(w0, xc[nt][0], bb)));
            }
        if constexpr (STORE) {
#pragma unroll
            for (int nt = 0; nt < NT; ++nt)
                if (h == 0 && pcol[nt] >= 0)
                    for (int c = 0; c < m.d; ++c)
                        sink.act[sink.act_off[0] + (long long)c * sink.P + pcol[nt]] =
                            (typename PR::Store)xc[nt][c];
        }
    }

    // ---------------- layers 2..L
    for (int l = 2; l <= L; ++l) {
        constexpr int NS = W / KPS;  // k-steps without bias
        Op bin[NT][NS];
#pragma unroll
        for (int nt = 0; nt < NT; ++nt) {
#pragma unroll
            for (int s = 0; s < NS; ++s) {
                if constexpr (BF) {
#pragma unroll
                    for (int p = 0; p < 8; ++p) {
                        const float z = acc[nt][s / 2][8 * (s % 2) + p];
                        bin[nt][s][p] = (__bf16)act_fn<ACT>(z, m.omega0);
                    }
                } else {
                    const float z = acc[nt][s / 16][s % 16];
                    bin[nt][s] = act_fn<ACT>(z, m.omega0);
                }
            }
            if constexpr (STORE) {
                // a_{l-1} (natural row order) for the weight gradients, and
                // its ReLU mask bits (SIREN: the derivative factors)
                if (pcol[nt] >= 0) {
                    // 32-bit element offsets: a per-lane part kept opaque so the
                    // per-row parts stay scalar (row constant x uniform stride)
                    const int P = (int)sink.P;
                    int base = (int)sink.act_off[l - 1] + pcol[nt] + 4 * h * P;
                    asm volatile("" : "+v"(base));
#pragma unroll
                    for (int mt = 0; mt < MT; ++mt)
#pragma unroll
                        for (int r = 0; r < 16; ++r) {
                            const float z = acc[nt][mt][r];
                            sink.act[base + (32 * mt + 8 * (r / 4) + (r % 4)) * P] =
                                (typename PR::Store)act_fn<ACT>(z, m.omega0);
                        }
                    if constexpr (ACT == INRCT_SIREN) {
                        int sb = (int)sink.sig_off[l - 1] + pcol[nt] + 4 * h * P;
                        asm volatile("" : "+v"(sb));
#pragma unroll
                        for (int mt = 0; mt < MT; ++mt)
#pragma unroll
                            for (int r = 0; r < 16; ++r)
                                sink.sig[sb + (32 * mt + 8 * (r / 4) + (r % 4)) * P] =
                                    act_grad<ACT>(acc[nt][mt][r], m.omega0);
                    } else {
                        sink.mask[((long long)(l - 2) * (sink.P / 32) + pcol[nt] / 32) * 64 + lane] =
                            relu_bits<MT>(acc[nt]);
                    }
                }
            }
        }
#pragma unroll
        for (int nt = 0; nt < NT; ++nt)
#pragma unroll
            for (int mt = 0; mt < MT; ++mt) acc[nt][mt] = (f32x16){0};
        const int KS = NS + 1;
        const Op *fr = frag + m.off[l] * 64;
#pragma unroll
        for (int mt = 0; mt < MT; ++mt) {
#pragma unroll
            for (int s = 0; s < NS; ++s) {
                const Op a = fr[((long long)s * MT + mt) * 64 + lane];
#pragma unroll
                for (int nt = 0; nt < NT; ++nt) acc[nt][mt] = PR::mma(a, bin[nt][s], acc[nt][mt]);
            }
            const Op a = fr[((long long)NS * MT + mt) * 64 + lane];
#pragma unroll
            for (int nt = 0; nt < NT; ++nt) acc[nt][mt] = PR::mma(a, one_b, acc[nt][mt]);
        }
    }
}

// f = w_out . act(z_L) + b_out for the lane's point (both halves combined).
template <int W, int NT, int ACT>
__device__ __forceinline__ void mlp_output(const MlpDev &m, const f32x16 (&acc)[NT][W / 32],
                                           float (&f)[NT]) {
    const int lane = threadIdx.x & 63;
    const int h = lane >> 5;
#pragma unroll
    for (int nt = 0; nt < NT; ++nt) {
        float s = 0.f;
#pragma unroll
        for (int mt = 0; mt < W / 32; ++mt)
#pragma unroll
            for (int r = 0; r < 16; ++r)
                s = fmaf(m.w_out[32 * mt + crow(r, h)], act_fn<ACT>(acc[nt][mt][r], m.omega0), s);
        s += __shfl_xor(s, 32);
        f[nt] = s + m.b_out[0];
    }
}

__device__ __forceinline__ float grid_coord(int i, int N) {
    return (float)(2 * i + 1 - N) / (float)N;
}

// ------------------------------------------------------- E on the grid
// Each wave evaluates 32*NT consecutive FOV ranks.
template <int W, int NT, bool BF, int ACT>
__global__ __launch_bounds__(256) void k_eval_grid(MlpDev m, long long n, float *__restrict__ u) {
    const int lane = threadIdx.x & 63;
    const int wave = threadIdx.x >> 6;
    const long long base = ((long long)blockIdx.x * 4 + wave) * (32 * NT);
    if (base >= n) return;
    float xc[NT][3];
    long long gidx[NT];
    int pcol[NT];
#pragma unroll
    for (int nt = 0; nt < NT; ++nt) {
        long long q = base + nt * 32 + (lane & 31);
        const bool ok = q < n;
        if (!ok) q = n - 1;
        int ix, iy, iz;
        gidx[nt] = fov_rank_to_index(m.fov, q, &ix, &iy, &iz);
        if (!ok) gidx[nt] = -1;
        xc[nt][0] = grid_coord(ix, m.fov.N);
        xc[nt][1] = grid_coord(iy, m.fov.N);
        xc[nt][2] = m.fov.dim == 3 ? grid_coord(iz, m.fov.N) : 0.f;
        pcol[nt] = -1;
    }
    f32x16 acc[NT][W / 32];
    ActSink<BF> sink{};
    mlp_forward<W, NT, BF, ACT, false>(m, xc, acc, sink, pcol);
    float f[NT];
    mlp_output<W, NT, ACT>(m, acc, f);
#pragma unroll
    for (int nt = 0; nt < NT; ++nt)
        if (lane < 32 && gidx[nt] >= 0) u[gidx[nt]] = f[nt];
}

// zero every grid point outside the FOV
__global__ void k_zero_outside(FovDev f, float *__restrict__ u, long long ngrid) {
    const long long t = (long long)blockIdx.x * 256 + threadIdx.x;
    if (t >= ngrid) return;
    const int x = (int)(t % f.N);
    const int y = (int)((t / f.N) % f.N);
    const int cnt = f.row_start[y + 1] - f.row_start[y];
    const int lo = f.xlo[y];
    if (x < lo || x >= lo + cnt) u[t] = 0.f;
}

__device__ __forceinline__ void index_coords(const FovDev &f, long long g, float *xc) {
    const int N = f.N;
    const int ix = (int)(g % N), iy = (int)((g / N) % N), iz = (int)(g / ((long long)N * N));
    xc[0] = grid_coord(ix, N);
    xc[1] = grid_coord(iy, N);
    xc[2] = f.dim == 3 ? grid_coord(iz, N) : 0.f;
}

// f at listed grid indices
template <int W, int NT, bool BF, int ACT>
__global__ __launch_bounds__(256) void k_eval_points(MlpDev m, const int32_t *__restrict__ idx,
                                                     long long k, float *__restrict__ out) {
    const int lane = threadIdx.x & 63;
    const int wave = threadIdx.x >> 6;
    const long long base = ((long long)blockIdx.x * 4 + wave) * (32 * NT);
    if (base >= k) return;
    float xc[NT][3];
    long long j[NT];
    int pcol[NT];
#pragma unroll
    for (int nt = 0; nt < NT; ++nt) {
        j[nt] = base + nt * 32 + (lane & 31);
        const long long jj = j[nt] < k ? j[nt] : k - 1;
        index_coords(m.fov, idx[jj], xc[nt]);
        pcol[nt] = -1;
    }
    f32x16 acc[NT][W / 32];
    ActSink<BF> sink{};
    mlp_forward<W, NT, BF, ACT, false>(m, xc, acc, sink, pcol);
    float f[NT];
    mlp_output<W, NT, ACT>(m, acc, f);
#pragma unroll
    for (int nt = 0; nt < NT; ++nt)
        if (lane < 32 && j[nt] < k) out[j[nt]] = f[nt];
}

// ---------------------------------------- E with LDS-staged weights (BF16)
// Persistent workgroups of four waves; a workgroup tile is 256 consecutive
// FOV ranks and each wave evaluates 64 of them (two 32-point N-tiles, so
// every A fragment read from LDS feeds two MFMAs).  The packed weights are
// one stream of "chunks" (one k-step of one layer: MT fragments of 1 KB,
// s-major), copied global -> LDS with direct-to-LDS loads kRingD chunks
// ahead into a ring of kRingD + 1 slots.  At each chunk boundary a wave
// waits until only its own later copies are outstanding, then the
// workgroup barrier makes the chunk visible and frees the slot the next
// copy overwrites.  The Fourier encoding uses the hardware sine/cosine on
// the fractional phase (turns), adequate for BF16 operands.
constexpr int kRingD = 6;
constexpr int kRingNB = kRingD + 1;

// 16-byte-per-lane copy global -> LDS (lane i lands at base + 16 i).  Issued
// from inline assembly: the compiler would otherwise assume every later LDS
// read may alias the copy and wait for all vector memory before it; here the
// ring protocol (explicit vmcnt wait + barrier) orders the accesses.  The
// instruction has no destination register; its address operand is read at
// issue.
__device__ __forceinline__ void dma16(const void *g, void *lds_wave_base) {
    const unsigned lds = (unsigned)(size_t)(__attribute__((address_space(3))) void *)lds_wave_base;
    asm volatile("s_mov_b32 m0, %0\n\tglobal_load_lds_dwordx4 %1, off"
                 :
                 : "s"(__builtin_amdgcn_readfirstlane(lds)), "v"(g)
                 : "memory", "m0");
}

template <int W>
struct RingCfg {
    static constexpr int MT = W / 32;
    static constexpr int PER_WAVE = MT / 4;           // fragment copies per wave per chunk
    static constexpr int CHUNK = MT * 1024;           // bytes
};

template <int W>
__device__ __forceinline__ void ring_issue(const char *__restrict__ gfrag, int chunk_src,
                                           char *ring, int slot, int wave, int lane) {
    typedef RingCfg<W> RC;
#pragma unroll
    for (int i = 0; i < RC::PER_WAVE; ++i) {
        const int f = wave * RC::PER_WAVE + i;
        const char *src = gfrag + ((size_t)chunk_src * RC::MT + f) * 1024 + lane * 16;
        dma16(src, ring + slot * RC::CHUNK + f * 1024);
    }
}

template <int W>
__device__ __forceinline__ void ring_wait() {
    // all but this wave's copies of the next kRingD - 1 chunks have landed
    if constexpr (RingCfg<W>::PER_WAVE == 2) asm volatile("s_waitcnt vmcnt(10)" ::: "memory");
    else asm volatile("s_waitcnt vmcnt(5)" ::: "memory");
}

template <int ACT>
__device__ __forceinline__ float act_bf(float z, float w0) {
    if constexpr (ACT == INRCT_FFN) return fmaxf(z, 0.f);
    else return __builtin_amdgcn_sinf(__builtin_amdgcn_fractf(w0 * z * 0.15915494309189535f));
}

// max(z, 0) in one instruction (no NaN canonicalisation of z first)
__device__ __forceinline__ float relu1(float z) {
    float r;
    asm("v_max_f32 %0, 0, %1" : "=v"(r) : "v"(z));
    return r;
}

// Eight accumulator values -> activated BF16 operand.  ReLU is applied after
// rounding, on the BF16 bit patterns as signed 16-bit integers (negative
// values, -0 included, have the sign bit set); rounding is monotonic and
// keeps the sign, so this equals rounding the rectified value.
template <int ACT>
__device__ __forceinline__ bf16x8 act_pack8(const f32x16 &a, int base, float w0) {
    bf16x8 t;
    if constexpr (ACT == INRCT_FFN) {
        typedef float f32x2 __attribute__((ext_vector_type(2)));
        typedef __bf16 bf16x2 __attribute__((ext_vector_type(2)));
        typedef short s16x2 __attribute__((ext_vector_type(2)));
        uint4 w;
        unsigned *wp = (unsigned *)&w;
#pragma unroll
        for (int pp = 0; pp < 4; ++pp) {
            const f32x2 f = {a[base + 2 * pp], a[base + 2 * pp + 1]};
            s16x2 q = __builtin_bit_cast(s16x2, __builtin_convertvector(f, bf16x2));
            q = __builtin_elementwise_max(q, (s16x2)0);
            wp[pp] = __builtin_bit_cast(unsigned, q);
        }
        t = __builtin_bit_cast(bf16x8, w);
    } else {
#pragma unroll
        for (int p = 0; p < 8; ++p) t[p] = (__bf16)act_bf<ACT>(a[base + p], w0);
    }
    return t;
}

template <int W, int ACT>
__global__ __launch_bounds__(256) void k_eval_lds(MlpDev m, int n, int ntiles, int nchunks,
                                                   float *__restrict__ u) {
    typedef RingCfg<W> RC;
    constexpr int MT = RC::MT;
    constexpr int NT = 2;
    constexpr int NS = W / 16;
    __shared__ __attribute__((aligned(16))) char ring[kRingNB * RC::CHUNK];
    __shared__ float sB[3 * 512];
    __shared__ float sWout[W];
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6, h = lane >> 5;
    const char *gfrag = (const char *)m.frag;
    // constants to LDS
    if constexpr (ACT == INRCT_FFN) {
        for (int i = threadIdx.x; i < m.F * m.d; i += 256) sB[i] = m.B[i];
    }
    for (int i = threadIdx.x; i < W; i += 256) sWout[i] = m.w_out[i];
    const float b_out = m.b_out[0];
    bf16x8 one_b;
#pragma unroll
    for (int p = 0; p < 8; ++p) one_b[p] = (__bf16)((h == 0 && p == 0) ? 1.f : 0.f);

    // ring state: slot being consumed, slot and source of the next copy
    int slot = 0, fill_slot = kRingD % kRingNB, fill_src = kRingD % nchunks;
#pragma unroll
    for (int i = 0; i < kRingD; ++i) ring_issue<W>(gfrag, i % nchunks, ring, i, wave, lane);

    auto next_chunk = [&]() -> const bf16x8 * {
        ring_wait<W>();
        __syncthreads();
        ring_issue<W>(gfrag, fill_src, ring, fill_slot, wave, lane);
        fill_src = fill_src + 1 == nchunks ? 0 : fill_src + 1;
        fill_slot = fill_slot + 1 == kRingNB ? 0 : fill_slot + 1;
        // read the ring through an address the compiler cannot trace (the
        // copies into it are invisible to it), keeping reads after the barrier
        unsigned off = (unsigned)(size_t)(__attribute__((address_space(3))) char *)ring +
                       (unsigned)(slot * RC::CHUNK);
        asm volatile("" : "+v"(off));
        slot = slot + 1 == kRingNB ? 0 : slot + 1;
        return (const bf16x8 *)(__attribute__((address_space(3))) const bf16x8 *)(size_t)off;
    };

    for (int tile = blockIdx.x; tile < ntiles; tile += gridDim.x) {
        float xc[NT][3];
        int gidx[NT];
        const int base = tile * 256 + wave * 64;
#pragma unroll
        for (int nt = 0; nt < NT; ++nt) {
            int q = base + nt * 32 + (lane & 31);
            const bool ok = q < n;
            if (!ok) q = n - 1;
            int ix, iy, iz;
            gidx[nt] = (int)fov_rank_to_index(m.fov, q, &ix, &iy, &iz);
            if (!ok) gidx[nt] = -1;
            xc[nt][0] = grid_coord(ix, m.fov.N);
            xc[nt][1] = grid_coord(iy, m.fov.N);
            xc[nt][2] = m.fov.dim == 3 ? grid_coord(iz, m.fov.N) : 0.f;
        }
        f32x16 acc[NT][MT];
#pragma unroll
        for (int nt = 0; nt < NT; ++nt)
#pragma unroll
            for (int mt = 0; mt < MT; ++mt) acc[nt][mt] = (f32x16){0};
        // ---------------- layer 1
        if constexpr (ACT == INRCT_FFN) {
            const int KS1 = m.F / 8;  // k-steps without the bias step
            for (int s = 0; s < KS1; ++s) {
                bf16x8 b[NT];
#pragma unroll
                for (int q = 0; q < 4; ++q) {
                    const int f = 8 * s + 4 * h + q;
                    const float bx = sB[f * m.d], by = sB[f * m.d + 1];
                    const float bz = m.d == 3 ? sB[f * m.d + 2] : 0.f;
#pragma unroll
                    for (int nt = 0; nt < NT; ++nt) {
                        const float t = fmaf(bz, xc[nt][2], fmaf(by, xc[nt][1], bx * xc[nt][0]));
                        const float r = __builtin_amdgcn_fractf(t);
                        b[nt][2 * q] = (__bf16)__builtin_amdgcn_sinf(r);
                        b[nt][2 * q + 1] = (__bf16)__builtin_amdgcn_cosf(r);
                    }
                }
                const bf16x8 *A = next_chunk();
#pragma unroll
                for (int mt = 0; mt < MT; ++mt) {
                    const bf16x8 a = A[mt * 64 + lane];
#pragma unroll
                    for (int nt = 0; nt < NT; ++nt)
                        acc[nt][mt] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(a, b[nt], acc[nt][mt], 0, 0, 0);
                }
            }
            const bf16x8 *A = next_chunk();
#pragma unroll
            for (int mt = 0; mt < MT; ++mt) {
                const bf16x8 a = A[mt * 64 + lane];
#pragma unroll
                for (int nt = 0; nt < NT; ++nt)
                    acc[nt][mt] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(a, one_b, acc[nt][mt], 0, 0, 0);
            }
        } else {
#pragma unroll
            for (int mt = 0; mt < MT; ++mt)
#pragma unroll
                for (int r = 0; r < 16; ++r) {
                    const int o = 32 * mt + crow(r, h);
                    const float w0 = m.W1[o * m.d], w1 = m.W1[o * m.d + 1];
                    const float w2 = m.d == 3 ? m.W1[o * m.d + 2] : 0.f;
                    const float bb = m.b1[o];
#pragma unroll
                    for (int nt = 0; nt < NT; ++nt)
                        acc[nt][mt][r] = fmaf(w2, xc[nt][2], fmaf(w1, xc[nt][1], fmaf(w0, xc[nt][0], bb)));
                }
        }
        // ---------------- layers 2..L
        for (int l = 2; l <= m.L; ++l) {
            bf16x8 bin[NT][NS];
#pragma unroll
            for (int nt = 0; nt < NT; ++nt)
#pragma unroll
                for (int s = 0; s < NS; ++s)
#pragma unroll
                    for (int p = 0; p < 8; ++p)
                        bin[nt][s][p] = (__bf16)act_bf<ACT>(acc[nt][s / 2][8 * (s % 2) + p], m.omega0);
#pragma unroll
            for (int s = 0; s <= NS; ++s) {
                const bf16x8 *A = next_chunk();
#pragma unroll
                for (int mt = 0; mt < MT; ++mt) {
                    const bf16x8 a = A[mt * 64 + lane];
#pragma unroll
                    for (int nt = 0; nt < NT; ++nt)
                        acc[nt][mt] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(
                            a, s < NS ? bin[nt][s] : one_b, s == 0 ? (f32x16){0} : acc[nt][mt],
                            0, 0, 0);
                }
            }
        }
        // ---------------- output layer
#pragma unroll
        for (int nt = 0; nt < NT; ++nt) {
            float sacc = 0.f;
#pragma unroll
            for (int mt = 0; mt < MT; ++mt)
#pragma unroll
                for (int r = 0; r < 16; ++r)
                    sacc = fmaf(sWout[32 * mt + crow(r, h)], act_bf<ACT>(acc[nt][mt][r], m.omega0), sacc);
            sacc += __shfl_xor(sacc, 32);
            if (lane < 32 && gidx[nt] >= 0) u[gidx[nt]] = sacc + b_out;
        }
        // keep the copy counter exact: drain stores and copies in flight
        asm volatile("s_waitcnt vmcnt(0)" ::: "memory");
    }
    asm volatile("s_waitcnt vmcnt(0)" ::: "memory");
}

// ------------------------------------------------------------------------
// Width-256 BF16 grid evaluation.  A workgroup of eight waves (two per SIMD)
// evaluates a tile of 256 FOV points, one 32-point column tile per wave.  The
// weights stream through a ring of 32 KB chunks in LDS (copied straight from
// global memory to LDS); a chunk is four k-steps of layer 1 (eight M-tiles)
// or eight k-steps of one half (four M-tiles) of a hidden layer.  Every
// fragment read from LDS feeds one product per wave; two waves per SIMD hide
// each other's LDS, barrier and vector-unit time.  Biases initialise the
// accumulators (from LDS), so no k-step carries them and no chunk is padded.
constexpr int kRingWD = 3;                 // chunks in flight
constexpr int kChunkW = 32 * 1024;
constexpr int kFovLdsN = 1024;             // largest grid side of the LDS path

// D chunks in flight, D + 1 slots.
template <int D>
struct RingW {
    static constexpr int NB = D + 1;
    char *ring;
    const char *gfrag;
    int slot, fill_slot, fill_src, nchunks, wave, lane;
    unsigned lds0;          // LDS byte address of the ring (uniform)
    const char *gsrc;       // this lane's 16 bytes of this wave's first fragment
    __device__ __forceinline__ void issue(int src, int dst_slot) {
        // the LDS destination is uniform: computed once per copy in scalar
        // registers, no per-copy address-space conversion
        const unsigned m0 = lds0 + (unsigned)(dst_slot * kChunkW + wave * 4 * 1024);
        const char *g = gsrc + (size_t)src * 32 * 1024;
#pragma unroll
        for (int i = 0; i < 4; ++i)
            asm volatile("s_mov_b32 m0, %0\n\tglobal_load_lds_dwordx4 %1, off"
                         :
                         : "s"(m0 + i * 1024), "v"(g + i * 1024)
                         : "memory", "m0");
    }
    __device__ __forceinline__ void start(int n) {
        wave = __builtin_amdgcn_readfirstlane(wave);
        lds0 = __builtin_amdgcn_readfirstlane(
            (unsigned)(size_t)(__attribute__((address_space(3))) char *)ring);
        gsrc = gfrag + (size_t)wave * 4 * 1024 + lane * 16;
        nchunks = n;
        slot = 0;
        fill_slot = D % NB;
        fill_src = D % n;
#pragma unroll
        for (int i = 0; i < D; ++i) issue(i % n, i);
    }
    // Waits for the next chunk, then refills the slot every wave has finished
    // with (the barrier orders this wave's refill after the other waves'
    // reads of it and publishes the other waves' copies of the next chunk).
    __device__ __forceinline__ const bf16x8 *next() {
        // all but this wave's copies of the next D - 1 chunks have landed
        static_assert(D == 2 || D == 3, "ring depth");
        if constexpr (D == 3) asm volatile("s_waitcnt vmcnt(8)" ::: "memory");
        else asm volatile("s_waitcnt vmcnt(4)" ::: "memory");
        __syncthreads();
        issue(fill_src, fill_slot);
        fill_src = fill_src + 1 == nchunks ? 0 : fill_src + 1;
        fill_slot = fill_slot + 1 == NB ? 0 : fill_slot + 1;
        // read the ring through an address the compiler cannot trace, so no
        // read is hoisted above the wait and barrier (the copies are asm)
        unsigned off = (unsigned)(size_t)(__attribute__((address_space(3))) char *)ring +
                       (unsigned)(slot * kChunkW);
        asm volatile("" : "+v"(off));
        slot = slot + 1 == NB ? 0 : slot + 1;
        return (const bf16x8 *)(__attribute__((address_space(3))) const bf16x8 *)(size_t)off;
    }
};

__device__ __forceinline__ void load_frags4(const bf16x8 *A, int j, int lane, bf16x8 (&af)[4]) {
#pragma unroll
    for (int mt = 0; mt < 4; ++mt) af[mt] = A[(j * 4 + mt) * 64 + lane];
}

__device__ __forceinline__ void load_frags8(const bf16x8 *A, int j, int lane, bf16x8 (&af)[8]) {
#pragma unroll
    for (int mt = 0; mt < 8; ++mt) af[mt] = A[(j * 8 + mt) * 64 + lane];
}

// Accumulator rows of M-tile mt for this lane (crow order) from a bias row
// of 256 floats in LDS: four runs of four consecutive outputs.
__device__ __forceinline__ f32x16 bias_tile(const float *sb, int mt, int h) {
    f32x16 a;
#pragma unroll
    for (int j = 0; j < 4; ++j) {
        const float4 v = *(const float4 *)(sb + 32 * mt + 8 * j + 4 * h);
        a[4 * j] = v.x;
        a[4 * j + 1] = v.y;
        a[4 * j + 2] = v.z;
        a[4 * j + 3] = v.w;
    }
    return a;
}

// Frequency rows of layer-1 k-step s for this lane's half h: four rows
// (bx, by, bz, 0), bz = 0 in 2-D.
__device__ __forceinline__ void ffn_rows(const float4 *sB4, int s, int h, float4 (&bq)[4]) {
#pragma unroll
    for (int q = 0; q < 4; ++q) bq[q] = sB4[8 * s + 4 * h + q];
}

__device__ __forceinline__ void ffn_feat1(const float4 (&bq)[4], const float (&xc)[3],
                                          bf16x8 &b) {
#pragma unroll
    for (int q = 0; q < 4; ++q) {
        const float t = fmaf(bq[q].z, xc[2], fmaf(bq[q].y, xc[1], bq[q].x * xc[0]));
        const float r = __builtin_amdgcn_fractf(t);
        b[2 * q] = (__bf16)__builtin_amdgcn_sinf(r);
        b[2 * q + 1] = (__bf16)__builtin_amdgcn_cosf(r);
    }
}

// Layer-1 k-step for one column tile with the features of the following
// k-step computed between the products (frequency mt / 2 after odd mt).
__device__ __forceinline__ void layer1_w(const bf16x8 (&af)[8], const bf16x8 &b, f32x16 (&acc)[8],
                                         const float4 (&bq)[4], const float (&xc)[3],
                                         bf16x8 &nb) {
#pragma unroll
    for (int mt = 0; mt < 8; ++mt) {
        acc[mt] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(af[mt], b, acc[mt], 0, 0, 0);
        if (mt & 1) {
            const int q = mt >> 1;
            const float t = fmaf(bq[q].z, xc[2], fmaf(bq[q].y, xc[1], bq[q].x * xc[0]));
            const float r = __builtin_amdgcn_fractf(t);
            nb[2 * q] = (__bf16)__builtin_amdgcn_sinf(r);
            nb[2 * q + 1] = (__bf16)__builtin_amdgcn_cosf(r);
        }
        __builtin_amdgcn_sched_barrier(0);
    }
}

// One hidden-layer half (four M-tiles) for one column tile: sixteen k-steps
// in two chunks, fragments read one k-step ahead; the second chunk's
// barrier comes before the first chunk's last products.
struct NoSide {
    __device__ __forceinline__ void operator()(int) const {}
};

// side(s) runs after the products of k-step s are issued: vector work of an
// earlier half (conversions, the output layer) overlaps the matrix core.
template <int HALF, bool BIAS, class Ring, class Side = NoSide>
__device__ __forceinline__ void half_gemm_w(Ring &rs, const bf16x8 (&bin)[16], const float *sb,
                                            int h, f32x16 (&acc)[4], int lane,
                                            Side &&side = Side()) {
    // accumulators start at the bias (or at zero when there is none)
#pragma unroll
    for (int mt = 0; mt < 4; ++mt)
        acc[mt] = BIAS ? bias_tile(sb, 4 * HALF + mt, h) : (f32x16){0};
    const bf16x8 *A = rs.next();
    bf16x8 cur[4], nxt[4];
    load_frags4(A, 0, lane, cur);
#pragma unroll
    for (int s = 0; s < 16; ++s) {
        if (s + 1 < 16) {
            if ((s + 1) % 8 == 0) A = rs.next();
            load_frags4(A, (s + 1) % 8, lane, nxt);
        }
        __builtin_amdgcn_sched_barrier(0);
#pragma unroll
        for (int mt = 0; mt < 4; ++mt)
            acc[mt] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(cur[mt], bin[s], acc[mt], 0, 0, 0);
        side(s);
        __builtin_amdgcn_sched_barrier(0);
#pragma unroll
        for (int mt = 0; mt < 4; ++mt) cur[mt] = nxt[mt];
    }
}

// FOV rank -> grid index (as fov_rank_to_index) with the row tables in LDS.
__device__ __forceinline__ int fov_decode_lds(const int32_t *sRow, const int32_t *sXlo, int N,
                                              int n_slice, int q, int *ox, int *oy, int *oz) {
    const int z = q / n_slice;
    const int rem = q - z * n_slice;
    int lo = 0, hi = N;  // last y with row_start[y] <= rem
    while (hi - lo > 1) {
        const int mid = (lo + hi) >> 1;
        if (sRow[mid] <= rem) lo = mid; else hi = mid;
    }
    const int x = sXlo[lo] + (rem - sRow[lo]);
    *ox = x;
    *oy = lo;
    *oz = z;
    return (z * N + lo) * N + x;
}

template <int ACT>
__global__ __launch_bounds__(512) void k_eval_lds_w(MlpDev m, int n, int ntiles, int nchunks,
                                                    const char *__restrict__ gfrag,
                                                    float *__restrict__ u) {
    constexpr int MT = 8, NS = 16;
    __shared__ __attribute__((aligned(16))) char ring[(kRingWD + 1) * kChunkW];
    __shared__ float4 sB4[512];
    __shared__ __attribute__((aligned(16))) float sBias[kMaxDepth * 256];
    __shared__ float sWout[256];
    __shared__ int32_t sRow[kFovLdsN + 1], sXlo[kFovLdsN];
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6, h = lane >> 5;
    if constexpr (ACT == INRCT_FFN) {
        for (int f = threadIdx.x; f < m.F; f += 512)
            sB4[f] = make_float4(m.B[f * m.d], m.B[f * m.d + 1], m.d == 3 ? m.B[f * m.d + 2] : 0.f,
                                 0.f);
    } else {
        // SIREN layer 1 rows (w_x, w_y, w_z, b), w_z = 0 in 2-D
        for (int o = threadIdx.x; o < 256; o += 512)
            sB4[o] = make_float4(m.W1[o * m.d], m.W1[o * m.d + 1],
                                 m.d == 3 ? m.W1[o * m.d + 2] : 0.f, m.b1[o]);
    }
    for (int i = threadIdx.x; i < m.L * 256; i += 512)
        sBias[i] = m.theta[m.boff[1 + i / 256] + i % 256];
    for (int i = threadIdx.x; i < 256; i += 512) sWout[i] = m.w_out[i];
    // the FOV row tables, so that decoding a tile's ranks reads no global memory
    for (int i = threadIdx.x; i <= m.fov.N; i += 512) sRow[i] = m.fov.row_start[i];
    for (int i = threadIdx.x; i < m.fov.N; i += 512) sXlo[i] = m.fov.xlo[i];
    __syncthreads();
    const float b_out = m.b_out[0];
    const float w0 = m.omega0;

    RingW<kRingWD> rs{ring, gfrag, 0, 0, 0, 0, wave, lane, 0u, nullptr};
    rs.start(nchunks);

    for (int tile = blockIdx.x; tile < ntiles; tile += gridDim.x) {
        float xc[3];
        int gidx;
        {
            int q = tile * 256 + wave * 32 + (lane & 31);
            const bool ok = q < n;
            if (!ok) q = n - 1;
            int ix, iy, iz;
            gidx = fov_decode_lds(sRow, sXlo, m.fov.N, m.fov.n_slice, q, &ix, &iy, &iz);
            if (!ok) gidx = -1;
            xc[0] = grid_coord(ix, m.fov.N);
            xc[1] = grid_coord(iy, m.fov.N);
            xc[2] = m.fov.dim == 3 ? grid_coord(iz, m.fov.N) : 0.f;
        }
        bf16x8 bin[NS];
        {
            // ---------------- layer 1, all eight M-tiles
            f32x16 acc[MT];
            if constexpr (ACT == INRCT_FFN) {
                // chunks of four k-steps; fragments one k-step ahead, the next
                // chunk's barrier before this chunk's last products, features
                // of the next k-step between the products (the index is
                // clamped at the end, where the extra features go unused)
                const int KS1 = m.F / 8;  // a multiple of four here
                const int nch1 = KS1 / 4;
#pragma unroll
                for (int mt = 0; mt < MT; ++mt) acc[mt] = bias_tile(sBias, mt, h);
                bf16x8 b, cur[MT], nxt[MT];
                {
                    float4 q0[4];
                    ffn_rows(sB4, 0, h, q0);
                    ffn_feat1(q0, xc, b);
                }
                const bf16x8 *A = rs.next();
                load_frags8(A, 0, lane, cur);
                for (int c = 0; c < nch1; ++c) {
                    const bool more = c + 1 < nch1;
#pragma unroll
                    for (int j = 0; j < 4; ++j) {
                        const int s = 4 * c + j;
                        if (j < 3) {
                            load_frags8(A, j + 1, lane, nxt);
                        } else if (more) {
                            A = rs.next();
                            load_frags8(A, 0, lane, nxt);
                        }
                        float4 q[4];
                        ffn_rows(sB4, min(s + 1, KS1 - 1), h, q);
                        bf16x8 nb;
                        __builtin_amdgcn_sched_barrier(0);
                        layer1_w(cur, b, acc, q, xc, nb);
                        b = nb;
#pragma unroll
                        for (int mt = 0; mt < MT; ++mt) cur[mt] = nxt[mt];
                        __builtin_amdgcn_sched_barrier(0);
                    }
                }
            } else {
#pragma unroll
                for (int mt = 0; mt < MT; ++mt)
#pragma unroll
                    for (int r = 0; r < 16; ++r) {
                        const float4 c = sB4[32 * mt + crow(r, h)];
                        acc[mt][r] = fmaf(c.z, xc[2], fmaf(c.y, xc[1], fmaf(c.x, xc[0], c.w)));
                    }
            }
#pragma unroll
            for (int s2 = 0; s2 < NS; ++s2) bin[s2] = act_pack8<ACT>(acc[s2 / 2], 8 * (s2 % 2), w0);
        }
        // ---------------- layers 2..L-1, two halves each
        for (int l = 2; l < m.L; ++l) {
            const float *sb = sBias + (l - 1) * 256;
            bf16x8 lo[8];
            f32x16 acc0[4], acc1[4];
            half_gemm_w<0, true>(rs, bin, sb, h, acc0, lane);
            // half 0's outputs are converted between half 1's products
            half_gemm_w<1, true>(rs, bin, sb, h, acc1, lane, [&](int s) {
                if (s < 8) lo[s] = act_pack8<ACT>(acc0[s / 2], 8 * (s % 2), w0);
            });
#pragma unroll
            for (int s2 = 0; s2 < 8; ++s2)
                bin[8 + s2] = act_pack8<ACT>(acc1[s2 / 2], 8 * (s2 % 2), w0);
#pragma unroll
            for (int s2 = 0; s2 < 8; ++s2) bin[s2] = lo[s2];
        }
        // ---------------- last hidden layer L and the linear output
        float fout = 0.f;
        if (m.L >= 2) {
            const float *sb = sBias + (m.L - 1) * 256;
            f32x16 acc0[4], acc1[4];
            auto out4 = [&](const f32x16 (&acc)[4], int half, int s) {
                // four of the half's 64 outputs: M-tile s / 4, slots 4 (s % 4) ..
                const int mt = s / 4;
#pragma unroll
                for (int i = 0; i < 4; ++i) {
                    const int r = 4 * (s % 4) + i;
                    fout = fmaf(sWout[32 * (4 * half + mt) + crow(r, h)],
                                ACT == INRCT_FFN ? relu1(acc[mt][r]) : act_bf<ACT>(acc[mt][r], w0),
                                fout);
                }
            };
            half_gemm_w<0, true>(rs, bin, sb, h, acc0, lane);
            // half 0's output-layer terms between half 1's products
            half_gemm_w<1, true>(rs, bin, sb, h, acc1, lane, [&](int s) { out4(acc0, 0, s); });
#pragma unroll
            for (int s = 0; s < 16; ++s) out4(acc1, 1, s);
        } else {
#pragma unroll
            for (int s2 = 0; s2 < NS; ++s2)
#pragma unroll
                for (int p = 0; p < 8; ++p) {
                    const int r = 8 * (s2 % 2) + p;
                    fout = fmaf(sWout[32 * (s2 / 2) + crow(r, h)], (float)bin[s2][p], fout);
                }
        }
        const float sacc = fout + __shfl_xor(fout, 32);
        if (lane < 32 && gidx >= 0) u[gidx] = sacc + b_out;
        // no drain: an older store in flight only makes the next ring wait stricter
    }
    // the copies of the chunks never consumed land before the wave ends
    asm volatile("s_waitcnt vmcnt(0)" ::: "memory");
}

// ------------------------------------------------------------------------
// Width-256 BF16 VJP of the sampled points (FFN), Algorithm 1's
// g = (n/|I|) sum_i v_i grad_theta f(x_i) before the dW contraction.  A
// workgroup of eight waves (one 32-point column tile each) recomputes the
// forward pass of k_eval_lds_w at 256 listed points, storing every layer
// input a_0 .. a_L (BF16 rows of P points) and keeping the ReLU masks of
// layers 1 .. L-1 in LDS, then runs the backward pass
//   delta_L = c w_out . relu'(z_L),  delta_{l-1} = (W_l^T delta_l) . relu'(z_{l-1}),
// storing delta_1 .. delta_L and delta_out = c, where c = scale v_i.  The
// transposed weights follow the forward weights in one chunk stream through
// a ring of three 32 KB slots.
constexpr int kMaxDepthV = 6;
struct VjpOut {
    __bf16 *act;                      // a_0 .. a_L: act_off[l] + row * P + point
    __bf16 *dlt;                      // delta_l at (l - 1) W P, delta_out at dlt_out
    long long P;
    long long act_off[kMaxDepth + 2];
    long long dlt_out;
};

// Stores one operand's eight BF16 values of this lane's point.  Rows are
// urow(p) + 4 h: the lane part 4 h P is folded into the (opaque) base and the
// uniform parts urow(p) P stay scalar, so no per-store vector address is
// precomputed.  P times any row fits in 32 bits.
__device__ __forceinline__ void store_rows8(__bf16 *lane_base, const bf16x8 &v,
                                            const int (&urow)[8], int P) {
    unsigned long long b = (unsigned long long)lane_base;
    asm volatile("" : "+v"(b));
#pragma unroll
    for (int p = 0; p < 8; ++p) ((__bf16 *)b)[urow[p] * P] = v[p];
}

// Uniform row parts of k-step s2 for the chained layers:
// chain_feature(s2, h, p) = 16 s2 + 8 (p / 4) + p % 4 + 4 h.
__device__ __forceinline__ void chain_urows(int s2, int (&row)[8]) {
#pragma unroll
    for (int p = 0; p < 8; ++p) row[p] = 16 * s2 + 8 * (p / 4) + (p % 4);
}

// delta = acc . mask (64 slots of one half), packed as BF16 operands.
__device__ __forceinline__ void mask_pack(const f32x16 (&acc)[4], uint2 bits, int s2,
                                          bf16x8 &out) {
    const f32x16 &a = acc[s2 / 2];
    const unsigned w = (s2 / 2) < 2 ? bits.x : bits.y;
    const int sh = 16 * ((s2 / 2) & 1) + 8 * (s2 % 2);
#pragma unroll
    for (int p = 0; p < 8; ++p)
        out[p] = (__bf16)((w >> (sh + p)) & 1u ? a[8 * (s2 % 2) + p] : 0.f);
}

__device__ __forceinline__ uint2 relu_bits4(const f32x16 (&acc)[4]) {
    unsigned w[2] = {0u, 0u};
#pragma unroll
    for (int mt = 0; mt < 4; ++mt)
#pragma unroll
        for (int r = 0; r < 16; ++r) w[mt >> 1] |= (acc[mt][r] > 0.f ? 1u : 0u) << (16 * (mt & 1) + r);
    return make_uint2(w[0], w[1]);
}

__global__ __launch_bounds__(512) void k_vjp_w(MlpDev m, const int32_t *__restrict__ idx,
                                               long long k, long long j0,
                                               const float *__restrict__ v, int v_compact,
                                               float scale, int ntiles, int nchunks,
                                               const char *__restrict__ gfrag, VjpOut o) {
    constexpr int MT = 8, NS = 16;
    __shared__ __attribute__((aligned(16))) char ring[3 * kChunkW];
    __shared__ float4 sB4[512];
    __shared__ __attribute__((aligned(16))) float sBias[kMaxDepthV * 256];
    __shared__ float sWout[256];
    // ReLU masks of layers 1 .. L-1: [wave][layer - 1][half][lane]
    __shared__ uint2 sMask[8 * (kMaxDepthV - 1) * 2 * 64];
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6, h = lane >> 5;
    for (int f = threadIdx.x; f < m.F; f += 512)
        sB4[f] = make_float4(m.B[f * m.d], m.B[f * m.d + 1], m.d == 3 ? m.B[f * m.d + 2] : 0.f,
                             0.f);
    for (int i = threadIdx.x; i < m.L * 256; i += 512)
        sBias[i] = m.theta[m.boff[1 + i / 256] + i % 256];
    for (int i = threadIdx.x; i < 256; i += 512) sWout[i] = m.w_out[i];
    __syncthreads();
    const int P = (int)o.P;
    const int L = m.L;
    uint2 *msk = sMask + (size_t)wave * (kMaxDepthV - 1) * 2 * 64 + lane;

    RingW<2> rs{ring, gfrag, 0, 0, 0, 0, wave, lane, 0u, nullptr};
    rs.start(nchunks);

    for (int tile = blockIdx.x; tile < ntiles; tile += gridDim.x) {
        const int pcol = tile * 256 + wave * 32 + (lane & 31);
        const long long jg = j0 + pcol;
        const bool ok = jg < k;
        const long long jj = ok ? jg : k - 1;
        const long long g = idx[jj];
        float xc[3];
        index_coords(m.fov, g, xc);
        const float cot = ok ? scale * (v_compact ? v[jj] : v[g]) : 0.f;
        // this lane's point, rows 4 h apart from the uniform row parts
        __bf16 *actp = o.act + pcol + (long long)(4 * h) * P;
        __bf16 *actp0 = actp + o.act_off[0];
        bf16x8 bin[NS];
        {
            // ---------------- layer 1 (as k_eval_lds_w), storing the features
            f32x16 acc[MT];
            const int KS1 = m.F / 8;
            const int nch1 = KS1 / 4;
#pragma unroll
            for (int mt = 0; mt < MT; ++mt) acc[mt] = bias_tile(sBias, mt, h);
            bf16x8 b, cur[MT], nxt[MT];
            {
                float4 q0[4];
                ffn_rows(sB4, 0, h, q0);
                ffn_feat1(q0, xc, b);
            }
            const bf16x8 *A = rs.next();
            load_frags8(A, 0, lane, cur);
            for (int c = 0; c < nch1; ++c) {
                const bool more = c + 1 < nch1;
#pragma unroll
                for (int j = 0; j < 4; ++j) {
                    const int s = 4 * c + j;
                    {
                        int row[8];
#pragma unroll
                        for (int p = 0; p < 8; ++p) row[p] = 8 * s + p / 2 + ((p % 2) ? m.F : 0);
                        store_rows8(actp0, b, row, P);
                    }
                    if (j < 3) {
                        load_frags8(A, j + 1, lane, nxt);
                    } else if (more) {
                        A = rs.next();
                        load_frags8(A, 0, lane, nxt);
                    }
                    float4 q[4];
                    ffn_rows(sB4, min(s + 1, KS1 - 1), h, q);
                    bf16x8 nb;
                    __builtin_amdgcn_sched_barrier(0);
                    layer1_w(cur, b, acc, q, xc, nb);
                    b = nb;
#pragma unroll
                    for (int mt = 0; mt < MT; ++mt) cur[mt] = nxt[mt];
                    __builtin_amdgcn_sched_barrier(0);
                }
            }
            msk[0] = relu_bits4(*(const f32x16(*)[4]) & acc[0]);
            msk[64] = relu_bits4(*(const f32x16(*)[4]) & acc[4]);
#pragma unroll
            for (int s2 = 0; s2 < NS; ++s2) {
                bin[s2] = act_pack8<INRCT_FFN>(acc[s2 / 2], 8 * (s2 % 2), 0.f);
                int row[8];
                chain_urows(s2, row);
                store_rows8(actp + o.act_off[1], bin[s2], row, P);
            }
        }
        // ---------------- layers 2..L-1, two halves each
        for (int l = 2; l < L; ++l) {
            const float *sb = sBias + (l - 1) * 256;
            bf16x8 lo[8];
            {
                f32x16 acc[4];
                half_gemm_w<0, true>(rs, bin, sb, h, acc, lane);
                msk[(l - 1) * 128] = relu_bits4(acc);
#pragma unroll
                for (int s2 = 0; s2 < 8; ++s2) lo[s2] = act_pack8<INRCT_FFN>(acc[s2 / 2], 8 * (s2 % 2), 0.f);
            }
            {
                f32x16 acc[4];
                half_gemm_w<1, true>(rs, bin, sb, h, acc, lane);
                msk[(l - 1) * 128 + 64] = relu_bits4(acc);
#pragma unroll
                for (int s2 = 0; s2 < 8; ++s2)
                    bin[8 + s2] = act_pack8<INRCT_FFN>(acc[s2 / 2], 8 * (s2 % 2), 0.f);
            }
#pragma unroll
            for (int s2 = 0; s2 < 8; ++s2) bin[s2] = lo[s2];
#pragma unroll
            for (int s2 = 0; s2 < NS; ++s2) {
                int row[8];
                chain_urows(s2, row);
                store_rows8(actp + o.act_off[l], bin[s2], row, P);
            }
        }
        // ---------------- last hidden layer: a_L stored, delta_L formed
        bf16x8 dl[NS];
        {
            const float *sb = sBias + (L - 1) * 256;
            __bf16 *dp = o.dlt + (long long)(L - 1) * 256 * P + pcol + (long long)(4 * h) * P;
#pragma unroll
            for (int half = 0; half < 2; ++half) {
                f32x16 acc[4];
                if (half == 0) half_gemm_w<0, true>(rs, bin, sb, h, acc, lane);
                else half_gemm_w<1, true>(rs, bin, sb, h, acc, lane);
#pragma unroll
                for (int s2 = 0; s2 < 8; ++s2) {
                    const int sg = 8 * half + s2;
                    int row[8];
                    chain_urows(sg, row);
                    const bf16x8 a = act_pack8<INRCT_FFN>(acc[s2 / 2], 8 * (s2 % 2), 0.f);
                    store_rows8(actp + o.act_off[L], a, row, P);
                    bf16x8 d;
#pragma unroll
                    for (int p = 0; p < 8; ++p) {
                        const float z = acc[s2 / 2][8 * (s2 % 2) + p];
                        d[p] = (__bf16)(z > 0.f ? cot * sWout[row[p] + 4 * h] : 0.f);
                    }
                    dl[sg] = d;
                    store_rows8(dp, d, row, P);
                }
            }
        }
        if (h == 0) o.dlt[o.dlt_out + pcol] = (__bf16)cot;
        // ---------------- backward: delta_{l-1} = (W_l^T delta_l) . relu'(z_{l-1})
        for (int l = L; l >= 2; --l) {
            __bf16 *dp = o.dlt + (long long)(l - 2) * 256 * P + pcol + (long long)(4 * h) * P;
            bf16x8 nlo[8];
            {
                f32x16 acc[4];
                half_gemm_w<0, false>(rs, dl, nullptr, h, acc, lane);
                const uint2 bits = msk[(l - 2) * 128];
#pragma unroll
                for (int s2 = 0; s2 < 8; ++s2) {
                    mask_pack(acc, bits, s2, nlo[s2]);
                    int row[8];
                    chain_urows(s2, row);
                    store_rows8(dp, nlo[s2], row, P);
                }
            }
            {
                f32x16 acc[4];
                half_gemm_w<1, false>(rs, dl, nullptr, h, acc, lane);
                const uint2 bits = msk[(l - 2) * 128 + 64];
#pragma unroll
                for (int s2 = 0; s2 < 8; ++s2) {
                    mask_pack(acc, bits, s2, dl[8 + s2]);
                    int row[8];
                    chain_urows(8 + s2, row);
                    store_rows8(dp, dl[8 + s2], row, P);
                }
            }
#pragma unroll
            for (int s2 = 0; s2 < 8; ++s2) dl[s2] = nlo[s2];
        }
    }
    // the copies of the chunks never consumed land before the wave ends
    asm volatile("s_waitcnt vmcnt(0)" ::: "memory");
}

// The width-128 BF16 FFN variant is held to two waves per SIMD (its fragment
// reads otherwise take every register, leaving one wave per SIMD).
template <int W, int NT, bool BF, int ACT>
__global__ __launch_bounds__(256, (W <= 128 && NT == 1 && BF && ACT == INRCT_FFN) ? 2 : 1)
void k_vjp_tile(MlpDev m, const int32_t *__restrict__ idx, long long k, long long j0,
                const float *__restrict__ v, int v_compact, float scale, long long ncols,
                ActSink<BF> sink, typename Prec<BF>::Store *__restrict__ dlt,
                long long dlt_off_L1) {
    typedef Prec<BF> PR;
    typedef typename PR::Op Op;
    typedef typename PR::Store St;
    constexpr int MT = W / 32;
    constexpr int KPS = PR::KPS;
    constexpr int NS = W / KPS;
    const int lane = threadIdx.x & 63;
    const int h = lane >> 5;
    const int wave = threadIdx.x >> 6;
    const long long cbase = ((long long)blockIdx.x * 4 + wave) * (32 * NT);
    if (cbase >= ncols) return;
    float xc[NT][3];
    float cot[NT];
    int pcol[NT];
#pragma unroll
    for (int nt = 0; nt < NT; ++nt) {
        pcol[nt] = (int)(cbase + nt * 32 + (lane & 31));
        const long long jg = j0 + pcol[nt];
        const bool ok = jg < k;
        const long long jj = ok ? jg : k - 1;
        const long long g = idx[jj];
        index_coords(m.fov, g, xc[nt]);
        cot[nt] = ok ? scale * (v_compact ? v[jj] : v[g]) : 0.f;
    }
    f32x16 acc[NT][MT];
    mlp_forward<W, NT, BF, ACT, true>(m, xc, acc, sink, pcol);
    const int L = m.L;
    const long long P = sink.P;
    // dlt rows: layer l (1..L) at dlt + (l-1)*W*P, output layer at dlt_off_L1
    // ---- output layer: delta_{L+1} = cot; store a_L; delta_L in registers
#pragma unroll
    for (int nt = 0; nt < NT; ++nt) {
        if (h == 0) dlt[dlt_off_L1 + pcol[nt]] = (St)cot[nt];
        const int Pi = (int)P;
        int ab = (int)sink.act_off[L] + pcol[nt] + 4 * h * Pi;
        int db = (L - 1) * W * Pi + pcol[nt] + 4 * h * Pi;
        asm volatile("" : "+v"(ab), "+v"(db));
#pragma unroll
        for (int mt = 0; mt < MT; ++mt)
#pragma unroll
            for (int r = 0; r < 16; ++r) {
                const int row = 32 * mt + crow(r, h);
                const int ro = (32 * mt + 8 * (r / 4) + (r % 4)) * Pi;
                const float z = acc[nt][mt][r];
                sink.act[ab + ro] = (St)act_fn<ACT>(z, m.omega0);
                // delta_L = cot * w_out * act'(z_L)
                const float dl = cot[nt] * m.w_out[row] * act_grad<ACT>(z, m.omega0);
                acc[nt][mt][r] = dl;
                dlt[db + ro] = (St)dl;
            }
    }
    const Op *fragT = (const Op *)m.fragT;
    for (int l = L; l >= 2; --l) {
        Op bin[NT][NS];
#pragma unroll
        for (int nt = 0; nt < NT; ++nt)
#pragma unroll
            for (int s = 0; s < NS; ++s) {
                if constexpr (BF) {
#pragma unroll
                    for (int p = 0; p < 8; ++p) bin[nt][s][p] = (__bf16)acc[nt][s / 2][8 * (s % 2) + p];
                } else {
                    bin[nt][s] = acc[nt][s / 16][s % 16];
                }
            }
#pragma unroll
        for (int nt = 0; nt < NT; ++nt)
#pragma unroll
            for (int mt = 0; mt < MT; ++mt) acc[nt][mt] = (f32x16){0};
        const Op *fr = fragT + m.offT[l] * 64;
#pragma unroll
        for (int mt = 0; mt < MT; ++mt)
#pragma unroll
            for (int s = 0; s < NS; ++s) {
                const Op a = fr[((long long)s * MT + mt) * 64 + lane];
#pragma unroll
                for (int nt = 0; nt < NT; ++nt) acc[nt][mt] = PR::mma(a, bin[nt][s], acc[nt][mt]);
            }
        // delta_{l-1} = (W_l^T delta_l) * act'(z_{l-1})
#pragma unroll
        for (int nt = 0; nt < NT; ++nt) {
            uint4 bits = make_uint4(0, 0, 0, 0);
            if constexpr (ACT == INRCT_FFN)
                bits = sink.mask[((long long)(l - 2) * (P / 32) + pcol[nt] / 32) * 64 + lane];
            const int Pi = (int)P;
            int db = (l - 2) * W * Pi + pcol[nt] + 4 * h * Pi;
            int sb = (int)sink.sig_off[l - 1] + pcol[nt] + 4 * h * Pi;
            asm volatile("" : "+v"(db), "+v"(sb));
#pragma unroll
            for (int mt = 0; mt < MT; ++mt)
#pragma unroll
                for (int r = 0; r < 16; ++r) {
                    const int ro = (32 * mt + 8 * (r / 4) + (r % 4)) * Pi;
                    float g;
                    if constexpr (ACT == INRCT_FFN) g = mask_bit(bits, 16 * mt + r);
                    else g = sink.sig[sb + ro];
                    const float dl = acc[nt][mt][r] * g;
                    acc[nt][mt][r] = dl;
                    dlt[db + ro] = (St)dl;
                }
        }
    }
}

// ------------------------------------------------ VJP phase 2: dW GEMMs
// Tile table entry: layer, M rows (delta rows), R inputs (act rows; column R
// is the bias), tile origin.
struct GemmTile {
    long long dlt_off;   // element offset of delta_l rows
    long long act_off;   // element offset of a_{l-1} rows
    int M, R, tm, tn;    // rows, inputs, tile origin (rows, cols)
    long long theta_off; // parameter offset of layer l (W then b)
};

template <bool BF>
__global__ __launch_bounds__(256) void k_dw_gemm(const GemmTile *__restrict__ tiles,
                                                 const typename Prec<BF>::Store *__restrict__ dlt,
                                                 const typename Prec<BF>::Store *__restrict__ act,
                                                 long long P, long long ncols, int kslice,
                                                 int accumulate,
                                                 float *__restrict__ part, int ntiles) {
    typedef Prec<BF> PR;
    typedef typename PR::Op Op;
    typedef typename PR::Store St;
    constexpr int KPS = PR::KPS;
    const GemmTile T = tiles[blockIdx.x];
    const int ks = blockIdx.y;
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    const int h = lane >> 5, i = lane & 31;
    const int wm = wave >> 1, wn = wave & 1;
    const long long p0 = (long long)ks * kslice;
    long long p1 = p0 + kslice;
    if (p1 > ncols) p1 = ncols;
    f32x16 acc[2][2];
#pragma unroll
    for (int a = 0; a < 2; ++a)
#pragma unroll
        for (int b = 0; b < 2; ++b) acc[a][b] = (f32x16){0};
    int rows[2], cols[2];
#pragma unroll
    for (int a = 0; a < 2; ++a) {
        rows[a] = T.tm + wm * 64 + a * 32 + i;
        cols[a] = T.tn + wn * 64 + a * 32 + i;
    }
    for (long long p = p0; p < p1; p += KPS) {
        Op A[2], B[2];
#pragma unroll
        for (int a = 0; a < 2; ++a) {
            if constexpr (BF) {
                if (rows[a] < T.M)
                    A[a] = *(const Op *)(dlt + T.dlt_off + (long long)rows[a] * P + p + 8 * h);
                else
                    for (int q = 0; q < 8; ++q) A[a][q] = (__bf16)0.f;
                if (cols[a] < T.R)
                    B[a] = *(const Op *)(act + T.act_off + (long long)cols[a] * P + p + 8 * h);
                else
                    for (int q = 0; q < 8; ++q) B[a][q] = (__bf16)(cols[a] == T.R ? 1.f : 0.f);
            } else {
                A[a] = rows[a] < T.M ? dlt[T.dlt_off + (long long)rows[a] * P + p + h] : 0.f;
                B[a] = cols[a] < T.R ? act[T.act_off + (long long)cols[a] * P + p + h]
                                     : (cols[a] == T.R ? 1.f : 0.f);
            }
        }
#pragma unroll
        for (int a = 0; a < 2; ++a)
#pragma unroll
            for (int b = 0; b < 2; ++b) acc[a][b] = PR::mma(A[a], B[b], acc[a][b]);
    }
    float *out = part + ((long long)ks * ntiles + blockIdx.x) * (128 * 128);
#pragma unroll
    for (int a = 0; a < 2; ++a)
#pragma unroll
        for (int b = 0; b < 2; ++b)
#pragma unroll
            for (int r = 0; r < 16; ++r) {
                const int lr = wm * 64 + a * 32 + crow(r, h);
                const int lc = wn * 64 + b * 32 + i;
                float *o = out + lr * 128 + lc;
                *o = accumulate ? *o + acc[a][b][r] : acc[a][b][r];
            }
}

// grad[theta] = sum over k-slices (fixed order) of the tile partials
__global__ void k_dw_reduce(const GemmTile *__restrict__ tiles, const float *__restrict__ part,
                            int ntiles, int nks, float *__restrict__ grad) {
    const long long t = (long long)blockIdx.x * 256 + threadIdx.x;
    if (t >= (long long)ntiles * 16384) return;
    const int tile = (int)(t / 16384);
    const int e = (int)(t % 16384);
    const GemmTile T = tiles[tile];
    const int row = T.tm + e / 128, col = T.tn + e % 128;
    if (row >= T.M || col > T.R) return;
    float s = 0.f;
    for (int k = 0; k < nks; ++k) s += part[((long long)k * ntiles + tile) * 16384 + e];
    const long long dst = col < T.R ? T.theta_off + (long long)row * T.R + col
                                    : T.theta_off + (long long)T.M * T.R + row;
    grad[dst] = s;
}

// BF16 dW GEMMs with full-width tiles: a workgroup computes a 256 x 256
// block of one layer's weight gradient (delta rows x input columns) over one
// slice of points, so every delta and activation row of the slice is read
// once per column block (layers of width 256 have one block).  The tile that
// starts at column 0 also sums the delta rows (the bias gradient).  Four
// waves, each a 128 x 128 quadrant (4 x 4 MFMA tiles).  The slice streams in
// groups of 32 points: a group is 16 delta and 16 activation fragments of
// 1 KB (256 rows x 16 points), copied straight from global memory into a
// ring of four 32 KB LDS slots, three groups in flight (each wave copies
// eight fragments and waits on its own copy counter; a barrier publishes the
// group), so every row is read from memory once per workgroup.
struct GemmTile2 {
    long long dlt_off;    // element offset of delta_l rows
    long long act_off;    // element offset of a_{l-1} rows
    long long theta_off;  // parameter offset of layer l (W then b)
    int M, R, tn, bias;   // rows, inputs, first column, sums the bias gradient
    int tw;               // columns the tile covers (its width: 256 or 128)
};
constexpr int kDwPart = 256 * 256 + 256;  // partial floats per (tile, slice)

// dW = delta A^T for one tile of TILE x TILE (256, or 128 for width-128
// MLPs, whose layers a 256-wide tile would cover a quarter of) over one
// slice of points.  Four waves, each (TILE / 64)^2 products of 32 x 32;
// partials are stored in the 256-stride layout either way.
template <int TILE>
__global__ __launch_bounds__(256) void k_dw_gemm2(const GemmTile2 *__restrict__ tiles,
                                                  const __bf16 *__restrict__ dlt,
                                                  const __bf16 *__restrict__ act, long long P,
                                                  long long ncols, int kslice, int accumulate,
                                                  float *__restrict__ part, int ntiles) {
    constexpr int MA = TILE / 64;        // 32-row (and 32-column) blocks per wave
    constexpr int FG = TILE / 8;         // fragments per group of 32 points
    constexpr int NC = FG / 4;           // copies per wave per group
    constexpr int SLOT = FG * 1024;
    __shared__ __attribute__((aligned(16))) char ring[4 * SLOT];
    const GemmTile2 T = tiles[blockIdx.x];
    const int ks = blockIdx.y;
    const int lane = threadIdx.x & 63;
    const int wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
    const int h = lane >> 5, i = lane & 31;
    const int wm = wave >> 1, wn = wave & 1;
    const long long p0 = (long long)ks * kslice;
    long long p1 = p0 + kslice;
    if (p1 > ncols) p1 = ncols;
    const int G = p1 > p0 ? (int)((p1 - p0) / 32) : 0;
    f32x16 acc[MA][MA];
#pragma unroll
    for (int a = 0; a < MA; ++a)
#pragma unroll
        for (int b = 0; b < MA; ++b) acc[a][b] = (f32x16){0};
    float bs[MA];
#pragma unroll
    for (int a = 0; a < MA; ++a) bs[a] = 0.f;
    const bool dob = T.bias && wn == 0;
    if (G > 0) {
        // fragment f of a group (lane l: row 32 (f / 2 % (TILE / 32)) + l % 32,
        // points 16 (f % 2) + 8 (l / 32) .. + 7): f < FG / 2 delta rows,
        // f >= FG / 2 activation rows of this tile's columns.  Rows past the
        // layer read its last row (their products are never summed into a
        // gradient).
        const __bf16 *src[NC];
#pragma unroll
        for (int q = 0; q < NC; ++q) {
            const int f = NC * wave + q;
            const int fr = f < FG / 2 ? f : f - FG / 2;
            const int row = 32 * ((fr >> 1) % (TILE / 32)) + i, off = 16 * (fr & 1) + 8 * h;
            if (f < FG / 2) src[q] = dlt + T.dlt_off + (long long)min(row, T.M - 1) * P + p0 + off;
            else src[q] = act + T.act_off + (long long)min(T.tn + row, T.R - 1) * P + p0 + off;
        }
        const unsigned lds0 = __builtin_amdgcn_readfirstlane(
            (unsigned)(size_t)(__attribute__((address_space(3))) char *)ring);
        // copies of group g (clamped to the last, so that every wave issues
        // the same number of copies per group whatever G is)
        auto issue = [&](int g, int slot) {
            const long long dp = 32LL * (g < G ? g : G - 1);
#pragma unroll
            for (int q = 0; q < NC; ++q)
                asm volatile("s_mov_b32 m0, %0\n\tglobal_load_lds_dwordx4 %1, off"
                             :
                             : "s"(lds0 + (unsigned)(slot * SLOT + (NC * wave + q) * 1024)),
                               "v"(src[q] + dp)
                             : "memory", "m0");
        };
        issue(0, 0);
        issue(1, 1);
        issue(2, 2);
        for (int g = 0; g < G; ++g) {
            // this wave's copies of group g have landed (those of g + 1 and
            // g + 2 may be in flight); the barrier publishes every wave's
            if constexpr (NC == 8) asm volatile("s_waitcnt vmcnt(16)" ::: "memory");
            else asm volatile("s_waitcnt vmcnt(8)" ::: "memory");
            __syncthreads();
            // the slot read through an address the compiler cannot trace, so
            // no read is hoisted above the wait and barrier
            unsigned off = (unsigned)(size_t)(__attribute__((address_space(3))) char *)ring +
                           (unsigned)((g & 3) * SLOT) + lane * 16;
            asm volatile("" : "+v"(off));
            const bf16x8 *F = (const bf16x8 *)(__attribute__((address_space(3))) const bf16x8 *)(size_t)off;
            bf16x8 A[2][MA], B[2][MA];
#pragma unroll
            for (int j = 0; j < 2; ++j)
#pragma unroll
                for (int a = 0; a < MA; ++a) {
                    A[j][a] = F[(((wm * MA + a) << 1) | j) * 64];
                    B[j][a] = F[(FG / 2 + (((wn * MA + a) << 1) | j)) * 64];
                }
            // the slot of group g - 1 is free (every wave passed this
            // barrier): group g + 3 goes there
            issue(g + 3, (g + 3) & 3);
#pragma unroll
            for (int j = 0; j < 2; ++j)
#pragma unroll
                for (int a = 0; a < MA; ++a)
#pragma unroll
                    for (int b = 0; b < MA; ++b)
                        acc[a][b] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(A[j][a], B[j][b],
                                                                            acc[a][b], 0, 0, 0);
            if (dob) {
#pragma unroll
                for (int a = 0; a < MA; ++a)
#pragma unroll
                    for (int j = 0; j < 2; ++j)
#pragma unroll
                        for (int q = 0; q < 8; ++q) bs[a] += (float)A[j][a][q];
            }
        }
        // the copies of the groups never consumed land before the wave ends
        asm volatile("s_waitcnt vmcnt(0)" ::: "memory");
    }
    float *__restrict__ out = part + ((long long)ks * ntiles + blockIdx.x) * kDwPart;
#pragma unroll
    for (int a = 0; a < MA; ++a)
#pragma unroll
        for (int b = 0; b < MA; ++b) {
            // rows crow(r, h) = 8 (r / 4) + 4 h + r % 4 of the 32-row tile
            float *o = out + (wm * (TILE / 2) + 32 * a + 4 * h) * 256 + wn * (TILE / 2) + 32 * b + i;
            if (accumulate) {
                // all sixteen earlier partials in flight before any store
                float prev[16];
#pragma unroll
                for (int r = 0; r < 16; ++r) prev[r] = o[(8 * (r / 4) + (r % 4)) * 256];
#pragma unroll
                for (int r = 0; r < 16; ++r) acc[a][b][r] += prev[r];
            }
#pragma unroll
            for (int r = 0; r < 16; ++r) o[(8 * (r / 4) + (r % 4)) * 256] = acc[a][b][r];
        }
    if (dob) {
#pragma unroll
        for (int a = 0; a < MA; ++a) {
            const float t = bs[a] + __shfl_xor(bs[a], 32);
            if (h == 0) {
                float *o = out + 256 * 256 + wm * (TILE / 2) + 32 * a + i;
                *o = accumulate ? *o + t : t;
            }
        }
    }
}

// grad[theta] = sum over slices (fixed order) of the full-width partials
__global__ void k_dw_reduce2(const GemmTile2 *__restrict__ tiles, const float *__restrict__ part,
                             int ntiles, int nks, float *__restrict__ grad) {
    const long long t = (long long)blockIdx.x * 256 + threadIdx.x;
    if (t >= (long long)ntiles * kDwPart) return;
    const int tile = (int)(t / kDwPart);
    const int e = (int)(t % kDwPart);
    const GemmTile2 T = tiles[tile];
    long long dst;
    if (e < 256 * 256) {
        const int row = e / 256, col = T.tn + e % 256;
        if (row >= T.M || col >= T.R || e % 256 >= T.tw) return;
        dst = T.theta_off + (long long)row * T.R + col;
    } else {
        const int row = e - 256 * 256;
        if (!T.bias || row >= T.M) return;
        dst = T.theta_off + (long long)T.M * T.R + row;
    }
    float s = 0.f;
    for (int k = 0; k < nks; ++k) s += part[((long long)k * ntiles + tile) * kDwPart + e];
    grad[dst] = s;
}

}  // namespace inrct

// ==================================================================== host
using namespace inrct;

namespace inrct {

static MlpDev make_dev(const inrct_model *m, const float *theta, const float *B) {
    MlpDev d{};
    d.kind = m->arch.kind;
    d.d = m->arch.in_dim;
    d.F = m->arch.n_freq;
    d.W = m->arch.width;
    d.L = m->arch.depth;
    d.omega0 = m->arch.omega0;
    d.frag = m->frag.ptr;
    d.fragT = m->fragT.ptr;
    const int L = m->arch.depth;
    d.w_out = theta + m->loff[L + 1];
    d.b_out = theta + m->loff[L + 1] + m->arch.width;
    d.W1 = theta + m->loff[1];
    d.b1 = theta + m->loff[1] + (long long)m->arch.in_dim * m->arch.width;
    d.B = B;
    for (int l = 0; l < 10 && l < kMaxDepth + 2; ++l) {
        d.off[l] = m->frag_off[l];
        d.offT[l] = m->fragT_off[l];
    }
    d.theta = theta;
    for (int l = 0; l < kMaxDepth + 2; ++l) d.boff[l] = 0;
    for (int l = 1; l <= L; ++l)
        d.boff[l] = m->loff[l] + (long long)layer_K(m->arch.kind, m->arch.n_freq,
                                                    m->arch.in_dim, m->arch.width, l) *
                                     m->arch.width;
    d.fov = m->fov.dev(m->dim);
    return d;
}

void model_pack(inrct_model *m, const float *theta, hipStream_t s) {
    if (m->arch.kind == INRCT_HASH) return;  // reads theta directly
    const MlpDev d = make_dev(m, theta, nullptr);
    const int slots = m->bf16() ? 8 : 1;
    const long long total = (m->nfrag + m->nfragT) * 64 * slots;
    if (total == 0) return;
    hipLaunchKernelGGL(k_pack, dim3((unsigned)cdiv(total, 256)), dim3(256), 0, s, d, theta,
                       m->bf16() ? 1 : 0, m->frag.ptr, m->fragT.ptr, m->nfrag, m->nfragT,
                       m->d_loff.as<long long>(), m->pk_layer.as<int>(), m->pk_mt.as<int>(),
                       m->pk_s.as<int>());
    INRCT_CHECK_LAUNCH();
    if (m->vjp_lds) {
        const long long tv = (m->nfrag_h + m->nfrag_vb) * 64 * 8;
        hipLaunchKernelGGL(k_pack, dim3((unsigned)cdiv(tv, 256)), dim3(256), 0, s, d, theta, 1,
                           m->frag_v.ptr, (char *)m->frag_v.ptr + m->nfrag_h * 64 * 16,
                           m->nfrag_h, m->nfrag_vb, m->d_loff.as<long long>(),
                           m->pkv_layer.as<int>(), m->pkv_mt.as<int>(), m->pkv_s.as<int>());
        INRCT_CHECK_LAUNCH();
    }
    if (m->nfrag_h > 0) {
        const long long th = m->nfrag_h * 64 * 8;
        hipLaunchKernelGGL(k_pack, dim3((unsigned)cdiv(th, 256)), dim3(256), 0, s, d, theta, 1,
                           m->frag_h.ptr, nullptr, m->nfrag_h, 0LL, m->d_loff.as<long long>(),
                           m->pkh_layer.as<int>(), m->pkh_mt.as<int>(), m->pkh_s.as<int>());
        INRCT_CHECK_LAUNCH();
    }
}

template <int W, int NT, bool BF, int ACT>
static void launch_eval_grid(const MlpDev &d, long long n, float *u, hipStream_t s) {
    const long long per_block = 4LL * 32 * NT;
    hipLaunchKernelGGL((k_eval_grid<W, NT, BF, ACT>), dim3((unsigned)cdiv(n, per_block)), dim3(256),
                       0, s, d, n, u);
    INRCT_CHECK_LAUNCH();
}

template <int W, int NT, bool BF, int ACT>
static void launch_eval_points(const MlpDev &d, const int32_t *idx, long long k, float *out,
                               hipStream_t s) {
    const long long per_block = 4LL * 32 * NT;
    hipLaunchKernelGGL((k_eval_points<W, NT, BF, ACT>), dim3((unsigned)cdiv(k, per_block)),
                       dim3(256), 0, s, d, idx, k, out);
    INRCT_CHECK_LAUNCH();
}

#define INRCT_DISPATCH_ACT(m, FN, W_, BF_, ...)                                \
    do {                                                                       \
        if ((m)->arch.kind == INRCT_FFN) FN<W_, 1, BF_, INRCT_FFN>(__VA_ARGS__);  \
        else FN<W_, 1, BF_, INRCT_SIREN>(__VA_ARGS__);                         \
    } while (0)

#define INRCT_DISPATCH_W_BF(m, FN, ...)                                        \
    do {                                                                       \
        if ((m)->arch.width == 256) {                                          \
            if ((m)->bf16()) INRCT_DISPATCH_ACT(m, FN, 256, true, __VA_ARGS__); \
            else INRCT_DISPATCH_ACT(m, FN, 256, false, __VA_ARGS__);           \
        } else {                                                               \
            if ((m)->bf16()) INRCT_DISPATCH_ACT(m, FN, 128, true, __VA_ARGS__); \
            else INRCT_DISPATCH_ACT(m, FN, 128, false, __VA_ARGS__);           \
        }                                                                      \
    } while (0)

void model_zero_outside(inrct_model *m, float *u, hipStream_t s) {
    hipLaunchKernelGGL(k_zero_outside, dim3((unsigned)cdiv(m->n_grid, 256)), dim3(256), 0, s,
                       m->fov.dev(m->dim), u, m->n_grid);
    INRCT_CHECK_LAUNCH();
}

template <int W, int ACT>
static void launch_eval_lds(const inrct_model *m, const MlpDev &d, float *u, hipStream_t s) {
    const long long ntiles = cdiv(m->n_fov, 256);
    long long nchunks = 0;
    const int l_first = m->arch.kind == INRCT_FFN ? 1 : 2;
    for (int l = l_first; l <= m->arch.depth; ++l)
        nchunks += ksteps(layer_K(m->arch.kind, m->arch.n_freq, m->arch.in_dim, W, l), 16);
    const long long grid = std::min<long long>(ntiles, m->n_cu);
    hipLaunchKernelGGL((k_eval_lds<W, ACT>), dim3((unsigned)grid), dim3(256), 0, s, d,
                       (int)m->n_fov, (int)ntiles, (int)nchunks, u);
    INRCT_CHECK_LAUNCH();
}

void model_eval_fov(inrct_model *m, const float *theta, const float *B, float *u,
                    hipStream_t s) {
    if (m->arch.kind == INRCT_HASH) {
        hash_eval(m, theta, nullptr, m->n_fov, u, s);
        return;
    }
    const MlpDev d = make_dev(m, theta, B);
    const bool lds_path = m->bf16() &&
                          (m->arch.kind != INRCT_FFN ||
                           (m->arch.n_freq <= 512 &&
                            (m->arch.width == 128 || m->arch.n_freq % 32 == 0))) &&
                          (m->arch.kind == INRCT_FFN || m->arch.depth >= 2) &&
                          m->N <= kFovLdsN;
    if (lds_path) {
        if (m->arch.width == 256) {
            const long long ntiles = cdiv(m->n_fov, 256);
            const long long grid = std::min<long long>(ntiles, m->n_cu);
            const int nchunks = (int)(m->nfrag_h / 32);
            if (m->arch.kind == INRCT_FFN)
                hipLaunchKernelGGL(k_eval_lds_w<INRCT_FFN>, dim3((unsigned)grid), dim3(512), 0, s,
                                   d, (int)m->n_fov, (int)ntiles, nchunks,
                                   (const char *)m->frag_h.ptr, u);
            else
                hipLaunchKernelGGL(k_eval_lds_w<INRCT_SIREN>, dim3((unsigned)grid), dim3(512), 0,
                                   s, d, (int)m->n_fov, (int)ntiles, nchunks,
                                   (const char *)m->frag_h.ptr, u);
            INRCT_CHECK_LAUNCH();
        } else {
            if (m->arch.kind == INRCT_FFN) launch_eval_lds<128, INRCT_FFN>(m, d, u, s);
            else launch_eval_lds<128, INRCT_SIREN>(m, d, u, s);
        }
        return;
    }
    INRCT_DISPATCH_W_BF(m, launch_eval_grid, d, m->n_fov, u, s);
}

void model_eval_grid(inrct_model *m, const float *theta, const float *B, float *u,
                     hipStream_t s, bool pack) {
    if (pack) model_pack(m, theta, s);
    model_zero_outside(m, u, s);
    model_eval_fov(m, theta, B, u, s);
}

static void model_eval_points(inrct_model *m, const float *theta, const float *B,
                              const int32_t *idx, long long k, float *out, hipStream_t s) {
    if (m->arch.kind == INRCT_HASH) {
        hash_eval(m, theta, idx, k, out, s);
        return;
    }
    model_pack(m, theta, s);
    const MlpDev d = make_dev(m, theta, B);
    INRCT_DISPATCH_W_BF(m, launch_eval_points, d, idx, k, out, s);
}

template <int W, int NT, bool BF, int ACT>
static void launch_vjp_chunk(inrct_model *m, const MlpDev &d, const int32_t *idx, long long k,
                             long long j0, long long ncols, const float *v, int v_compact,
                             float scale, int accumulate, hipStream_t s) {
    typedef typename Prec<BF>::Store St;
    ActSink<BF> sink{};
    sink.act = m->act.as<St>();
    sink.sig = m->sig.as<float>();
    sink.P = m->P_alloc;
    sink.mask = m->mask.as<uint4>();
    for (int l = 0; l < 10 && l < kMaxDepth + 2; ++l) {
        sink.act_off[l] = m->act_off[l];
        sink.sig_off[l] = m->sig_off[l];
    }
    const long long P = m->P_alloc;
    const long long dlt_L1 = (long long)m->arch.depth * m->arch.width * P;
    if (BF && W == 256 && ACT == INRCT_FFN && m->vjp_lds) {
        VjpOut o{};
        o.act = m->act.as<__bf16>();
        o.dlt = m->dlt.as<__bf16>();
        o.P = P;
        for (int l = 0; l < kMaxDepth + 2; ++l) o.act_off[l] = m->act_off[l];
        o.dlt_out = dlt_L1;
        const int ntiles = (int)cdiv(ncols, 256);
        const int grid = (int)std::min<long long>(ntiles, m->n_cu);
        const int nchunks = (int)((m->nfrag_h + m->nfrag_vb) / 32);
        hipLaunchKernelGGL(k_vjp_w, dim3((unsigned)grid), dim3(512), 0, s, d, idx, k, j0, v,
                           v_compact, scale, ntiles, nchunks, (const char *)m->frag_v.ptr, o);
    } else {
        const long long per_block = 4LL * 32 * NT;
        hipLaunchKernelGGL((k_vjp_tile<W, NT, BF, ACT>), dim3((unsigned)cdiv(ncols, per_block)),
                           dim3(256), 0, s, d, idx, k, j0, v, v_compact, scale, ncols, sink,
                           m->dlt.as<St>(), dlt_L1);
    }
    INRCT_CHECK_LAUNCH();
    if constexpr (BF)
        if (m->dw_tile == 128)
            hipLaunchKernelGGL(k_dw_gemm2<128>, dim3(m->ntiles, m->nks), dim3(256), 0, s,
                               m->tiles.as<GemmTile2>(), (const __bf16 *)m->dlt.ptr,
                               (const __bf16 *)m->act.ptr, P, ncols, m->kslice, accumulate,
                               m->part.as<float>(), m->ntiles);
        else
            hipLaunchKernelGGL(k_dw_gemm2<256>, dim3(m->ntiles, m->nks), dim3(256), 0, s,
                               m->tiles.as<GemmTile2>(), (const __bf16 *)m->dlt.ptr,
                               (const __bf16 *)m->act.ptr, P, ncols, m->kslice, accumulate,
                               m->part.as<float>(), m->ntiles);
    else
        hipLaunchKernelGGL((k_dw_gemm<BF>), dim3(m->ntiles, m->nks), dim3(256), 0, s,
                           m->tiles.as<GemmTile>(), (const St *)m->dlt.ptr, (const St *)m->act.ptr,
                           P, ncols, m->kslice, accumulate, m->part.as<float>(), m->ntiles);
    INRCT_CHECK_LAUNCH();
}

void model_vjp(inrct_model *m, const float *theta, const float *B, const int32_t *idx,
               long long k, const float *v, int v_compact, double scale, float *grad,
               hipStream_t s, bool pack) {
    if (m->arch.kind == INRCT_HASH) {
        hash_vjp(m, theta, idx, k, v, v_compact, scale, grad, s);
        return;
    }
    if (pack) model_pack(m, theta, s);
    const MlpDev d = make_dev(m, theta, B);
    const long long P = m->P_alloc;
    int chunk = 0;
    for (long long j0 = 0; j0 < k; j0 += P, ++chunk) {
        long long ncols = k - j0 < P ? k - j0 : P;
        ncols = cdiv(ncols, 256) * 256;  // P is a multiple of 256
        if (ncols > P) ncols = P;
        INRCT_DISPATCH_W_BF(m, launch_vjp_chunk, m, d, idx, k, j0, ncols, v, v_compact,
                            (float)scale, chunk > 0 ? 1 : 0, s);
    }
    if (m->bf16())
        hipLaunchKernelGGL(k_dw_reduce2, dim3((unsigned)cdiv((long long)m->ntiles * kDwPart, 256)),
                           dim3(256), 0, s, m->tiles.as<GemmTile2>(), m->part.as<float>(),
                           m->ntiles, m->nks, grad);
    else
        hipLaunchKernelGGL(k_dw_reduce, dim3((unsigned)cdiv((long long)m->ntiles * 16384, 256)),
                           dim3(256), 0, s, m->tiles.as<GemmTile>(), m->part.as<float>(),
                           m->ntiles, m->nks, grad);
    INRCT_CHECK_LAUNCH();
}

}  // namespace inrct

namespace inrct {
// Argument checks of inrct_model_create.
void check_model_args(const inr_arch *arch, const inr_grid *grid, int64_t max_k) {
    INRCT_REQUIRE(arch && grid, "null argument");
    const inr_arch &a = *arch;
    INRCT_REQUIRE(grid->dim == 2 || grid->dim == 3, "grid dim must be 2 or 3");
    INRCT_REQUIRE(grid->n >= 1 && grid->n <= 4096, "grid n must be in [1, 4096]");
    INRCT_REQUIRE(a.in_dim == grid->dim, "arch in_dim must equal the grid dim");
    INRCT_REQUIRE(a.kind == INRCT_FFN || a.kind == INRCT_SIREN || a.kind == INRCT_HASH,
                  "unknown INR kind %d", a.kind);
    if (a.kind == INRCT_HASH) {
        INRCT_REQUIRE(a.width == 16 || a.width == 32 || a.width == 64,
                      "hash INR width must be 16, 32 or 64");
        INRCT_REQUIRE(a.depth >= 1 && a.depth <= kHashMaxDepth && a.width * a.depth <= 128,
                      "hash INR needs 1 <= depth <= 4 and width * depth <= 128");
        INRCT_REQUIRE(a.mlp_dtype == INRCT_FP32, "hash INR runs in FP32");
        INRCT_REQUIRE(a.hash_levels >= 1 && a.hash_levels <= kHashMaxLevels,
                      "hash levels must be in [1, %d]", kHashMaxLevels);
        INRCT_REQUIRE(a.hash_log2_size >= 4 && a.hash_log2_size <= 24,
                      "hash table size must be 2^4 .. 2^24");
        INRCT_REQUIRE(a.hash_base_res >= 1 && a.hash_max_res >= a.hash_base_res &&
                          a.hash_max_res <= (1 << 20),
                      "hash resolutions must satisfy 1 <= base <= max <= 2^20");
    } else {
        INRCT_REQUIRE(a.width == 128 || a.width == 256, "width must be 128 or 256");
        INRCT_REQUIRE(a.depth >= 1 && a.depth <= kMaxDepth, "depth must be in [1, %d]",
                      kMaxDepth);
    }
    INRCT_REQUIRE(a.mlp_dtype == INRCT_FP32 || a.mlp_dtype == INRCT_BF16, "unknown mlp dtype");
    if (a.kind == INRCT_FFN)
        INRCT_REQUIRE(a.n_freq >= 8 && a.n_freq % 8 == 0 && a.n_freq <= 4096,
                      "FFN needs n_freq a positive multiple of 8");
    INRCT_REQUIRE(max_k >= 1, "max_k must be >= 1");
}

// Everything a model handle holds on the device, carved from `ar` (arch, N,
// dim and max_k already set).  Run once to size the workspace and once to
// carve it.
void build_model(inrct_model *m, Arena &ar) {
    const inr_arch &a = m->arch;
    m->n_grid = 1;
    for (int i = 0; i < m->dim; ++i) m->n_grid *= m->N;
    INRCT_REQUIRE(m->n_grid < (1LL << 31), "grid too large for int32 indices");
    m->fov.build(ar, m->dim, m->N);
    {
        // compute units of the current device (they size the dW split); with
        // no device (sizing on a host without a GPU) an MI355X's 256
        int dev = 0, ncu = 0;
        if (hipGetDevice(&dev) != hipSuccess ||
            hipDeviceGetAttribute(&ncu, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess)
            ncu = 0;
        (void)hipGetLastError();
        m->n_cu = ncu > 0 ? ncu : 256;
    }
    m->n_fov = m->fov.n;
    INRCT_REQUIRE(m->n_fov >= 1, "empty FOV");
    m->max_k = std::min<long long>(m->max_k, m->n_fov);
    if (a.kind == INRCT_HASH) {
        hash_setup(m, ar);
        // sampler scratch and Adam partials, as below
        m->flags.alloc(ar, (size_t)m->n_fov);
        m->n_blk = cdiv(m->n_fov, 4096);
        m->blk.alloc(ar, (size_t)(m->n_blk + 1) * sizeof(int64_t));
        m->n_apart = adam_partials(m->n_params);
        m->apart.alloc(ar, sizeof(double) * m->n_apart);
        return;
    }
    const int W = a.width, L = a.depth, d = a.in_dim;
    const bool bf = a.mlp_dtype == INRCT_BF16;
    const int kps = bf ? 16 : 2;
    // parameter offsets
    m->loff.assign(L + 2, 0);
    long long off = 0;
    for (int l = 1; l <= L + 1; ++l) {
        m->loff[l] = off;
        const int K = l == L + 1 ? W : layer_K(a.kind, a.n_freq, d, W, l);
        const int O = l == L + 1 ? 1 : W;
        off += (long long)K * O + O;
    }
    m->n_params = off;
    upload(ar, m->d_loff, m->loff);
    // fragment tables
    std::vector<int> fl, fm, fs;
    const int MT = W / 32;
    const int l_first = a.kind == INRCT_FFN ? 1 : 2;
    for (int l = l_first; l <= L; ++l) {
        const int KS = ksteps(layer_K(a.kind, a.n_freq, d, W, l), kps);
        m->frag_off[l] = (long long)fl.size();
        for (int s = 0; s < KS; ++s)
            for (int mt = 0; mt < MT; ++mt) {
                fl.push_back(l);
                fm.push_back(mt);
                fs.push_back(s);
            }
    }
    m->nfrag = (long long)fl.size();
    for (int l = 2; l <= L; ++l) {
        const int NS = W / kps;
        m->fragT_off[l] = (long long)fl.size() - m->nfrag;
        for (int s = 0; s < NS; ++s)
            for (int mt = 0; mt < MT; ++mt) {
                fl.push_back(l);
                fm.push_back(mt);
                fs.push_back(s);
            }
    }
    m->nfragT = (long long)fl.size() - m->nfrag;
    if (bf && W == 256) {
        // chunk stream of the width-256 LDS kernel (biases excluded):
        // layer 1 by k-step x 8 M-tiles, hidden layers by half, then
        // k-step x 4 M-tiles
        std::vector<int> hl, hm, hs;
        if (a.kind == INRCT_FFN) {
            const int KS1 = ksteps(layer_K(a.kind, a.n_freq, d, W, 1), 16) - 1;
            for (int s = 0; s < KS1; ++s)
                for (int mt = 0; mt < 8; ++mt) {
                    hl.push_back(1);
                    hm.push_back(mt);
                    hs.push_back(s);
                }
        }
        for (int l = 2; l <= L; ++l)
            for (int half = 0; half < 2; ++half)
                for (int s = 0; s < 16; ++s)
                    for (int mt = 0; mt < 4; ++mt) {
                        hl.push_back(l);
                        hm.push_back(half * 4 + mt);
                        hs.push_back(s);
                    }
        m->nfrag_h = (long long)hl.size();
        upload(ar, m->pkh_layer, hl);
        upload(ar, m->pkh_mt, hm);
        upload(ar, m->pkh_s, hs);
        m->frag_h.alloc(ar, m->nfrag_h * 64 * 16);
        m->vjp_lds = a.kind == INRCT_FFN && a.n_freq % 32 == 0 &&
                     a.n_freq <= 512 && L >= 2 && L <= kMaxDepthV;
        if (m->vjp_lds) {
            // backward stream: layers L .. 2, by half, k-step x 4 M-tiles
            // of W_l^T (M-tiles over the inputs of layer l)
            std::vector<int> vl = hl, vm = hm, vs = hs;
            for (int l = L; l >= 2; --l)
                for (int half = 0; half < 2; ++half)
                    for (int s = 0; s < 16; ++s)
                        for (int mt = 0; mt < 4; ++mt) {
                            vl.push_back(l);
                            vm.push_back(half * 4 + mt);
                            vs.push_back(s);
                        }
            m->nfrag_vb = (long long)vl.size() - m->nfrag_h;
            upload(ar, m->pkv_layer, vl);
            upload(ar, m->pkv_mt, vm);
            upload(ar, m->pkv_s, vs);
            m->frag_v.alloc(ar, (m->nfrag_h + m->nfrag_vb) * 64 * 16);
        }
    }
    upload(ar, m->pk_layer, fl);
    upload(ar, m->pk_mt, fm);
    upload(ar, m->pk_s, fs);
    const size_t fbytes = bf ? 16 : 4;
    m->frag.alloc(ar, std::max<long long>(1, m->nfrag) * 64 * fbytes);
    m->fragT.alloc(ar, std::max<long long>(1, m->nfragT) * 64 * fbytes);
    // VJP scratch: chunk of P_alloc points
    const long long kpad = cdiv(m->max_k, 256) * 256;
    m->P_alloc = std::min<long long>(kpad, 262144);
    m->nks = (int)cdiv(m->P_alloc, m->kslice);
    const long long P = m->P_alloc;
    const int K1 = layer_K(a.kind, a.n_freq, d, W, 1);
    m->act_off[0] = 0;
    for (int l = 1; l <= L; ++l) m->act_off[l] = (long long)K1 * P + (long long)(l - 1) * W * P;
    m->act_elems = (long long)K1 * P + (long long)L * W * P;
    m->dlt_elems = (long long)L * W * P + P;
    const size_t es = bf ? 2 : 4;
    m->act.alloc(ar, m->act_elems * es);
    m->mask.alloc(ar, sizeof(uint4) * (size_t)std::max(1, L - 1) * (P / 32) * 64);
    m->dlt.alloc(ar, m->dlt_elems * es);
    if (a.kind == INRCT_SIREN) {
        for (int l = 1; l <= L; ++l) m->sig_off[l] = (long long)(l - 1) * W * P;
        m->sig_elems = (long long)L * W * P;
        m->sig.alloc(ar, m->sig_elems * sizeof(float));
    }
    if (bf) {
        // full-width dW tiles: layer l = 1..L+1, dw_tile input columns each
        // (128 for width-128 MLPs, whose layers fit one 128 x 128 tile)
        m->dw_tile = W <= 128 ? 128 : 256;
        std::vector<GemmTile2> tiles2;
        for (int l = 1; l <= L + 1; ++l) {
            GemmTile2 t{};
            t.M = l == L + 1 ? 1 : W;
            t.R = l == L + 1 ? W : layer_K(a.kind, a.n_freq, d, W, l);
            t.dlt_off = (long long)(l - 1) * W * P;
            t.act_off = m->act_off[l - 1];
            t.theta_off = m->loff[l];
            t.tw = m->dw_tile;
            for (int tn = 0; tn < t.R; tn += m->dw_tile) {
                GemmTile2 u = t;
                u.tn = tn;
                u.bias = tn == 0;
                tiles2.push_back(u);
            }
        }
        m->ntiles = (int)tiles2.size();
        upload(ar, m->tiles, tiles2);
        // split-K slices of 2048 points, shortened (to no less than
        // 512) when the chunk is too small to give every CU a block
        const long long want = cdiv((long long)m->n_cu, (long long)m->ntiles);
        const long long ks = cdiv(cdiv(P, want), 256) * 256;
        m->kslice = (int)std::min<long long>(2048, std::max<long long>(512, ks));
        m->nks = (int)cdiv(P, m->kslice);
        m->part.alloc(ar, (size_t)m->nks * m->ntiles * kDwPart * sizeof(float));
    }
    // dW GEMM tiles: layer l = 1..L+1, delta rows M, inputs R (+ bias col)
    std::vector<GemmTile> tiles;
    for (int l = 1; l <= L + 1; ++l) {
        GemmTile t{};
        t.M = l == L + 1 ? 1 : W;
        t.R = l == L + 1 ? W : layer_K(a.kind, a.n_freq, d, W, l);
        t.dlt_off = (long long)(l - 1) * W * P;
        t.act_off = m->act_off[l - 1];
        t.theta_off = m->loff[l];
        for (int tm = 0; tm < t.M; tm += 128)
            for (int tn = 0; tn <= t.R; tn += 128) {
                GemmTile u = t;
                u.tm = tm;
                u.tn = tn;
                tiles.push_back(u);
            }
    }
    if (!bf) {
        m->ntiles = (int)tiles.size();
        upload(ar, m->tiles, tiles);
        m->part.alloc(ar, (size_t)m->nks * m->ntiles * 16384 * sizeof(float));
    }
    // sampler scratch
    m->flags.alloc(ar, (size_t)m->n_fov);
    m->n_blk = cdiv(m->n_fov, 4096);
    m->blk.alloc(ar, (size_t)(m->n_blk + 1) * sizeof(int64_t));
    // Adam partials
    m->n_apart = adam_partials(m->n_params);
    m->apart.alloc(ar, sizeof(double) * m->n_apart);
}

inrct_model *fresh_model(const inr_arch *arch, const inr_grid *grid, int64_t max_k) {
    inrct_model *m = new inrct_model();
    m->arch = *arch;
    m->N = grid->n;
    m->dim = grid->dim;
    m->max_k = max_k;
    return m;
}
}  // namespace inrct

extern "C" {

int inrct_model_create(const inr_arch *arch, const inr_grid *grid, int64_t max_k, void *ws,
                       size_t ws_bytes, hipStream_t stream, inrct_model **out) {
    return guarded([&] {
        INRCT_REQUIRE(out, "null argument");
        *out = nullptr;
        check_model_args(arch, grid, max_k);
        inrct_model *m = fresh_model(arch, grid, max_k);
        try {
            build_in_workspace(
                m, m->ws, ws, ws_bytes, stream, [&] { return fresh_model(arch, grid, max_k); },
                [](inrct_model *h, Arena &ar) { build_model(h, ar); });
        } catch (...) {
            delete m;
            throw;
        }
        *out = m;
    });
}

int inrct_model_destroy(inrct_model *model) {
    delete model;
    return INRCT_OK;
}

int64_t inrct_model_n_params(const inrct_model *model) { return model ? model->n_params : -1; }
int64_t inrct_model_n_fov(const inrct_model *model) { return model ? model->n_fov : -1; }

int inr_eval_grid(inrct_model *model, const float *theta, const float *B, float *u,
                  hipStream_t stream) {
    return guarded([&] {
        INRCT_REQUIRE(model && theta && u, "null argument");
        INRCT_REQUIRE(model->arch.kind != INRCT_FFN || B, "FFN needs B");
        model_eval_grid(model, theta, B, u, stream);
    });
}

int inr_eval_points(inrct_model *model, const float *theta, const float *B, const int32_t *idx,
                    int64_t k, float *f_out, hipStream_t stream) {
    return guarded([&] {
        INRCT_REQUIRE(model && theta && (k == 0 || (idx && f_out)), "null argument");
        INRCT_REQUIRE(model->arch.kind != INRCT_FFN || B, "FFN needs B");
        INRCT_REQUIRE(k >= 0, "k must be >= 0");
        if (k > 0) model_eval_points(model, theta, B, idx, k, f_out, stream);
    });
}

int inr_vjp_subsampled(inrct_model *model, const float *theta, const float *B,
                       const int32_t *idx, int64_t k, const float *v, int v_compact,
                       double scale, float *grad, hipStream_t stream) {
    return guarded([&] {
        INRCT_REQUIRE(model && theta && idx && v && grad, "null argument");
        INRCT_REQUIRE(model->arch.kind != INRCT_FFN || B, "FFN needs B");
        INRCT_REQUIRE(k >= 1 && k <= model->max_k, "k must be in [1, max_k=%lld]",
                      (long long)model->max_k);
        model_vjp(model, theta, B, idx, k, v, v_compact, scale, grad, stream);
    });
}

}  // extern "C"
