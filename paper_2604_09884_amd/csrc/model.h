// Internal definition of the model handle (shared by mlp.hip and step.hip).
#pragma once

#include "geom.h"

namespace inrct {
constexpr int kHashMaxLevels = 32;  // hash encoding: levels per model
constexpr int kHashMaxDepth = 4;    // hash encoding: hidden layers
constexpr int kHashSlice = 256;     // hash VJP: points per dW partial sum
constexpr int kAdamMaxPartials = 1024;  // Adam: float64 partials of ||g||^2
}  // namespace inrct

struct inrct_model {
    inrct::Workspace ws;
    inr_arch arch;
    int N = 0, dim = 0;
    int n_cu = 256;  // compute units of the device the handle was created on
    long long n_grid = 0, n_params = 0, n_fov = 0, max_k = 0;
    inrct::FovHost fov;

    // parameter offsets of each affine layer (1-based; L+1 = output layer)
    std::vector<long long> loff;
    inrct::DevBuf d_loff;

    // packed MFMA A operands: forward (layers 1..L or 2..L) and transposed
    // (layers 2..L); one record per fragment: layer, M-tile, k-step
    long long nfrag = 0, nfragT = 0;
    long long frag_off[10] = {0}, fragT_off[10] = {0};
    inrct::DevBuf frag, fragT, pk_layer, pk_mt, pk_s;
    // chunk stream of the width-256 BF16 grid-evaluation kernel
    long long nfrag_h = 0;
    inrct::DevBuf frag_h, pkh_layer, pkh_mt, pkh_s;
    // chunk stream of the width-256 VJP kernel: the forward stream (nfrag_h
    // fragments, as frag_h) followed by nfrag_vb transposed fragments
    long long nfrag_vb = 0;
    inrct::DevBuf frag_v, pkv_layer, pkv_mt, pkv_s;
    bool vjp_lds = false;

    // VJP chunk scratch
    long long P_alloc = 0;       // points per chunk (row stride)
    int kslice = 2048, nks = 0;  // split-K slice length and count
    long long act_off[10] = {0}, sig_off[10] = {0};
    long long act_elems = 0, dlt_elems = 0, sig_elems = 0;
    inrct::DevBuf act, dlt, sig, part, tiles, mask;
    int ntiles = 0;
    int dw_tile = 256;           // BF16 dW tile width (128 for width-128 MLPs)

    // sampler: FOV-rank membership bytes and per-block counts
    inrct::DevBuf flags, blk;
    long long n_blk = 0;

    // Adam float64 partials
    inrct::DevBuf apart;
    int n_apart = 0;

    // hash encoding: level resolutions, per-point VJP rows, table-gradient
    // contributions (keys, positions, the sort's second key / position
    // buffers, values and sorted values), the sort's digit counts and dW
    // slice partials
    int hash_res[inrct::kHashMaxLevels] = {0};
    int hash_row = 0, hash_key_bits = 0;
    inrct::DevBuf hash_rows, hash_key, hash_pos, hash_skey, hash_spos, hash_val, hash_sval,
        hash_cnt, hash_part;

    bool bf16() const { return arch.mlp_dtype == INRCT_BF16; }
};

namespace inrct {
// sampler / Adam / E helpers implemented in mlp.hip and step.hip
void check_model_args(const inr_arch *arch, const inr_grid *grid, int64_t max_k);
inrct_model *fresh_model(const inr_arch *arch, const inr_grid *grid, int64_t max_k);
void build_model(inrct_model *m, Arena &ar);
void model_pack(inrct_model *m, const float *theta, hipStream_t s);
void model_eval_grid(inrct_model *m, const float *theta, const float *B, float *u,
                     hipStream_t s, bool pack = true);
void model_zero_outside(inrct_model *m, float *u, hipStream_t s);
void model_eval_fov(inrct_model *m, const float *theta, const float *B, float *u,
                    hipStream_t s);
void model_vjp(inrct_model *m, const float *theta, const float *B, const int32_t *idx,
               long long k, const float *v, int v_compact, double scale, float *grad,
               hipStream_t s, bool pack = true);
// hash-encoding INR (hash.hip)
void hash_setup(inrct_model *m, Arena &a);
void hash_eval(inrct_model *m, const float *theta, const int32_t *idx, long long n,
               float *out, hipStream_t s);
void hash_vjp(inrct_model *m, const float *theta, const int32_t *idx, long long k,
              const float *v, int v_compact, double scale, float *grad, hipStream_t s);
void model_sample(inrct_model *m, uint64_t seed, uint64_t step, long long k, int32_t *idx,
                  hipStream_t s);
int adam_partials(long long p);
void model_adam(inrct_model *m, float *theta, float *mm, float *vv, const float *g,
                long long t, double lr, double b1, double b2, double eps, double *gn2,
                hipStream_t s);

int64_t geom_rays(const inrct_geom *g);
int geom_dim(const inrct_geom *g);
int geom_N(const inrct_geom *g);
void backproject(inrct_geom *geom, const float *r, float *v, hipStream_t s);
void backproject_at(inrct_geom *geom, const float *r, const int32_t *idx, int64_t k,
                    float *out, hipStream_t s);
void residual_loss(inrct_geom *geom, int loss, const float *z, const float *y, float *r,
                   double *loss_out, hipStream_t s);
}  // namespace inrct
