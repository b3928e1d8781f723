// Learned-CDF form of the code sort.
//
// A small monotone network maps the top bits of a husky code to its
// approximate rank (a cumulative distribution), so that one pass can send
// every (code, index) pair near its final place: the sort becomes a bucket
// scatter plus independent sorts of small buckets.  The paper's coder is
// order-preserving (Sec. 3.2); the bucket function built here is made
// order-preserving too, which is what keeps the result exact:
//
//  * window: codes are clamped to [lo, hi] (the sample's range) and W = the
//    24 bits right below the common prefix of lo and hi, so W never
//    decreases as the code grows;
//  * network 1 -> 64 -> 64 -> 1, ReLU, every weight = softplus(parameter) > 0,
//    so its output never decreases in x = W / 2^24; trained in FP32 on a
//    seeded 1 % sample of codes (targets (rank + 0.5) / S) with mean squared
//    error and Adam, by the forward/backward/update kernels below;
//  * LUT[W] = network(W / 2^24) quantised to u32 for all 2^24 + 1 cell
//    starts, then a running maximum, so the table is monotone whatever the
//    network does (LUT[0] = 0, LUT[2^24] = 2^32 - 1);
//  * cell W owns buckets [b(W), b(W+1)), b(W) = LUT[W] * B >> 32.  A cell
//    owning two or more buckets splits its keys by equal-depth splitters
//    taken from the sorted sample (full 64-bit codes), so even a cell that
//    holds one heavy key prefix is spread over its share of buckets;
//  * bucket ids (16 bits, B = 65,536) drive two stable 8-bit LSD passes that
//    move (code, index, id); each bucket then holds its keys in input order,
//    and the segmented radix sort of radix.hip sorts every bucket by code:
//    buckets of at most one tile in LDS, larger ("overflowing") buckets by
//    its multi-tile passes.  Runs of equal codes never cross buckets, so the
//    fix-up that follows is the plain path's.

#include <hip/hip_ext.h>
#include <algorithm>
#include <cmath>

#include "../../include/husky.h"
#include "common.h"
#include "internal.h"
#include "bucket.h"
#include "rank.h"

namespace husky {

constexpr int HID = 64;
constexpr int NPARAM = HID + HID + HID * HID + HID + HID + 1;  // 4353
constexpr int O_V1 = 0, O_B1 = HID, O_V2 = 2 * HID, O_B2 = 2 * HID + HID * HID, O_V3 = O_B2 + HID,
              O_B3 = O_V3 + HID;
constexpr int MLP_T = 256;  // threads (and samples per round) of the training kernel

using LearnedHeader = husky_learned_header;
static_assert(sizeof(LearnedHeader) <= 256, "header fits its slot");

struct ModelView {
    LearnedHeader* hdr;
    float* params;
    float* adam_m;
    float* adam_v;
    uint32_t* lut;        // [LUT_CELLS + 1]
    uint64_t* splitters;  // [B]
    uint32_t* dense;      // [B / 2] dense cells, ascending
    uint32_t* dense_cum;  // [B / 2 + 1] dense sample keys in the dense cells before each
    uint16_t* subtab;     // [16 B] per heavy cell: header, then splitters below each sub-cell
    uint64_t* cellinfo;   // [2^24] buckets of every cell (and sub-cell keys of heavy ones)
};
constexpr uint32_t MAX_DENSE = LEARNED_BUCKETS / 2;
constexpr uint32_t DENSE_MIN = 16;

static size_t al256(size_t x) { return (x + 255) / 256 * 256; }

// Byte offsets of the model's parts (husky_learned_part order), then the total.
constexpr int N_PARTS = 10;
static void model_offsets(size_t off[N_PARTS + 1]) {
    size_t o = 0;
    const size_t sz[N_PARTS] = {256, NPARAM * 4, NPARAM * 4, NPARAM * 4, (size_t)(LUT_CELLS + 1) * 4,
                                (size_t)LEARNED_BUCKETS * 8, (size_t)MAX_DENSE * 4,
                                (size_t)(MAX_DENSE + 1) * 4, (size_t)LEARNED_BUCKETS * SUB_SLOT * 2,
                                (size_t)LUT_CELLS * 8};
    for (int i = 0; i < N_PARTS; ++i) {
        off[i] = o;
        o += al256(sz[i]);
    }
    off[N_PARTS] = o;
}

static ModelView model_view(void* model) {
    size_t off[N_PARTS + 1];
    model_offsets(off);
    uint8_t* p = (uint8_t*)model;
    ModelView m;
    m.hdr = (LearnedHeader*)(p + off[0]);
    m.params = (float*)(p + off[1]);
    m.adam_m = (float*)(p + off[2]);
    m.adam_v = (float*)(p + off[3]);
    m.lut = (uint32_t*)(p + off[4]);
    m.splitters = (uint64_t*)(p + off[5]);
    m.dense = (uint32_t*)(p + off[6]);
    m.dense_cum = (uint32_t*)(p + off[7]);
    m.subtab = (uint16_t*)(p + off[8]);
    m.cellinfo = (uint64_t*)(p + off[9]);
    return m;
}

typedef float f32x16 __attribute__((ext_vector_type(16)));  // one 32 x 32 fp32 MFMA block per lane

__device__ __forceinline__ float softplusf(float v) { return v > 20.f ? v : log1pf(expf(v)); }
__device__ __forceinline__ float sigmoidf(float v) { return 1.f / (1.f + expf(-v)); }

// Effective weight of a raw parameter: softplus for the monotone network,
// the raw value for the deliberately unconstrained one (fault injection).
template <bool MONO>
__device__ __forceinline__ float eff(float v) { return MONO ? softplusf(v) : v; }
template <bool MONO>
__device__ __forceinline__ float deff(float v) { return MONO ? sigmoidf(v) : 1.f; }

// SplitMix64 (Steele, Lea, Flood 2014): counter-based 64-bit generator.
__device__ __forceinline__ uint64_t splitmix64(uint64_t x) {
    x += 0x9E3779B97F4A7C15ull;
    x = (x ^ (x >> 30)) * 0xBF58476D1CE4E5B9ull;
    x = (x ^ (x >> 27)) * 0x94D049BB133111EBull;
    return x ^ (x >> 31);
}
__device__ __forceinline__ float unit_noise(uint64_t seed, uint64_t i) {  // in [-1, 1)
    return (float)((double)(splitmix64(seed * 0x100000001B3ull + i) >> 11) * (1.0 / 9007199254740992.0)) * 2.f - 1.f;
}

// ------------------------------------------------------------------ init
// Deterministic start: first-layer knots spread over [0, 1] (w1 ~ 1,
// b1 = -(j + 0.5) / 64), second layer ~ 1/64, output ~ 1/32, small seeded
// noise on every parameter; Adam moments zero.  The raw-weight network
// starts from the same function (its weights are the softplus values).
__global__ void k_mlp_init(float* params, float* m, float* v, uint64_t seed, int raw) {
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= NPARAM) return;
    const float e = 0.05f * unit_noise(seed, (uint64_t)i);
    float p;
    if (i < O_B1) p = 0.5413f + e;  // softplus^-1(1)
    else if (i < O_V2) p = -((float)(i - O_B1) + 0.5f) / HID + 0.1f * e;
    else if (i < O_B2) p = -4.15f + e;  // softplus^-1(1/64)
    else if (i < O_V3) p = 0.1f * e;
    else if (i < O_B3) p = -3.45f + e;  // softplus^-1(1/32)
    else p = 0.f;
    const bool weight = i < O_B1 || (i >= O_V2 && i < O_B2) || (i >= O_V3 && i < O_B3);
    if (raw && weight) p = softplusf(p);
    params[i] = p;
    m[i] = 0.f;
    v[i] = 0.f;
}

// ------------------------------------------------------------------ forward / backward
// One workgroup (four wavefronts) takes `per_block` consecutive samples of
// the batch, 32 per wavefront at a time, and writes the gradient of the
// batch's mean squared error, summed over its samples, to
// partial[block][NPARAM]; the loss sum goes to partial[block][NPARAM].  The
// three 64 x 64 products run on the matrix cores (v_mfma_f32_32x32x2f32: in
// an output block lane l holds row 8(v / 4) + 4(l / 32) + v % 4 and column
// l % 32 in register v; the A operand of a step is row l % 32 at column
// l / 32 of that step's pair, the B operand row l / 32 of the pair at
// column l % 32):
//   forward   z2^T = W2 h1^T      rows hidden unit k, columns the 32 samples;
//   weights   dW2 += dz2^T h1     K runs over the samples, accumulated in
//                                 registers for all of the wavefront's;
//   backward  dh1^T = W2^T dz2^T  rows hidden unit j, columns the samples.
// h1 is recomputed from x wherever an operand needs it; dz2, relu(z2) and
// dz1 pass through LDS ([sample][unit]) to change layout, and the vector
// gradients (dw3, db2, dw1, db1) are column sums over them, one unit per
// lane.  Wavefront partials are added in a fixed order, so the result does
// not depend on timing.
template <bool MONO>
__global__ __launch_bounds__(MLP_T) void k_mlp_grad(const float* __restrict__ params,
                                                    const float* __restrict__ xs,
                                                    const float* __restrict__ ys, uint32_t first,
                                                    uint32_t count, uint32_t stride,
                                                    uint32_t per_block, float inv_batch,
                                                    float* __restrict__ partial) {
    constexpr int NWV = MLP_T / WAVE;  // wavefronts
    constexpr int CH = 32;             // samples per wavefront step
    constexpr int LD = HID + 1;        // padded LDS row
    static_assert(NWV * HID * HID <= 2 * NWV * CH * LD, "wavefront dW2 partials fit the staging area");
    __shared__ float W2[HID * HID];  // effective weights [k][j]
    __shared__ float w1[HID], b1[HID], b2[HID], w3[HID];
    __shared__ float s_buf[2 * NWV * CH * LD];
    __shared__ float s_x[NWV][CH], s_g[NWV][CH];
    __shared__ float s_vec[NWV][6][HID];  // per wavefront: dw3, db2, dw1, db1, db3 / loss
    const uint32_t tid = threadIdx.x, w = tid / WAVE, l = lane_id(), half = l / 32, col = l % 32;
    float* s_dz = s_buf + w * CH * LD;             // dz2 as [sample][k]
    float* s_r = s_buf + (NWV + w) * CH * LD;      // relu(z2), then dz1, as [sample][unit]
    for (int i = tid; i < HID * HID; i += MLP_T) W2[i] = eff<MONO>(params[O_V2 + i]);
    if (tid < HID) {
        w1[tid] = eff<MONO>(params[O_V1 + tid]);
        b1[tid] = params[O_B1 + tid];
        b2[tid] = params[O_B2 + tid];
        w3[tid] = eff<MONO>(params[O_V3 + tid]);
    }
    const float b3 = params[O_B3];
    __syncthreads();
    // forward A operands (rows of W2) and the h1 coefficients this lane's
    // weight-gradient B operands use
    float a0[HID / 2], a1[HID / 2];
#pragma unroll
    for (int st = 0; st < HID / 2; ++st) {
        a0[st] = W2[(int)col * HID + 2 * st + (int)half];
        a1[st] = W2[(32 + (int)col) * HID + 2 * st + (int)half];
    }
    const float w1c0 = w1[col], b1c0 = b1[col], w1c1 = w1[32 + col], b1c1 = b1[32 + col];
    f32x16 gw00 = {}, gw01 = {}, gw10 = {}, gw11 = {};
    float acc_w3 = 0.f, acc_b2 = 0.f, acc_w1 = 0.f, acc_b1 = 0.f, acc_b3 = 0.f, acc_loss = 0.f;
    const uint32_t s0 = blockIdx.x * per_block;
    const uint32_t s1 = min(count, s0 + per_block);
    for (uint32_t base = s0; base < s1; base += NWV * CH) {  // uniform per workgroup
        const uint32_t smp = base + w * CH + col;
        const bool ok = smp < s1;
        const uint32_t src = first + smp * stride;
        const float x = ok ? xs[src] : 0.f;
        const float yv = ok ? ys[src] : 0.f;
        // forward
        f32x16 z0 = {}, z1 = {};
#pragma unroll
        for (int st = 0; st < HID / 2; ++st) {
            const int j = 2 * st + (int)half;
            const float h = fmaxf(w1[j] * x + b1[j], 0.f);
            z0 = __builtin_amdgcn_mfma_f32_32x32x2f32(a0[st], h, z0, 0, 0, 0);
            z1 = __builtin_amdgcn_mfma_f32_32x32x2f32(a1[st], h, z1, 0, 0, 0);
        }
        float part = 0.f;
#pragma unroll
        for (int v = 0; v < 16; ++v) {
            const int k = 8 * (v / 4) + 4 * (int)half + (v % 4);
            part += w3[k] * fmaxf(z0[v] + b2[k], 0.f) + w3[32 + k] * fmaxf(z1[v] + b2[32 + k], 0.f);
        }
        const float out = b3 + (part + __shfl_xor(part, 32, WAVE));
        const float d = ok ? out - yv : 0.f;
        const float g = 2.f * d * inv_batch;
        if (half == 0) {
            acc_loss += d * d;
            acc_b3 += g;
            s_x[w][col] = x;
            s_g[w][col] = g;
        }
#pragma unroll
        for (int v = 0; v < 16; ++v) {
            const int k = 8 * (v / 4) + 4 * (int)half + (v % 4);
            const float p0 = z0[v] + b2[k], p1 = z1[v] + b2[32 + k];
            s_dz[col * LD + k] = p0 > 0.f ? g * w3[k] : 0.f;
            s_dz[col * LD + 32 + k] = p1 > 0.f ? g * w3[32 + k] : 0.f;
            s_r[col * LD + k] = fmaxf(p0, 0.f);
            s_r[col * LD + 32 + k] = fmaxf(p1, 0.f);
        }
        __syncthreads();
        // dW2 += dz2^T h1 over the wavefront's 32 samples (two per step)
#pragma unroll
        for (int st = 0; st < CH / 2; ++st) {
            const int sm = 2 * st + (int)half;
            const float xsm = s_x[w][sm];
            const float az0 = s_dz[sm * LD + col], az1 = s_dz[sm * LD + 32 + col];
            const float h0 = fmaxf(w1c0 * xsm + b1c0, 0.f), h1v = fmaxf(w1c1 * xsm + b1c1, 0.f);
            gw00 = __builtin_amdgcn_mfma_f32_32x32x2f32(az0, h0, gw00, 0, 0, 0);
            gw01 = __builtin_amdgcn_mfma_f32_32x32x2f32(az0, h1v, gw01, 0, 0, 0);
            gw10 = __builtin_amdgcn_mfma_f32_32x32x2f32(az1, h0, gw10, 0, 0, 0);
            gw11 = __builtin_amdgcn_mfma_f32_32x32x2f32(az1, h1v, gw11, 0, 0, 0);
        }
        // dw3 and db2: lane l sums unit l over the samples
        for (int sm = 0; sm < CH; ++sm) {
            acc_w3 += s_g[w][sm] * s_r[sm * LD + l];
            acc_b2 += s_dz[sm * LD + l];
        }
        // dh1^T = W2^T dz2^T
        f32x16 dh0 = {}, dh1 = {};
#pragma unroll
        for (int st = 0; st < HID / 2; ++st) {
            const int k = 2 * st + (int)half;
            const float bz = s_dz[col * LD + k];
            dh0 = __builtin_amdgcn_mfma_f32_32x32x2f32(W2[k * HID + col], bz, dh0, 0, 0, 0);
            dh1 = __builtin_amdgcn_mfma_f32_32x32x2f32(W2[k * HID + 32 + col], bz, dh1, 0, 0, 0);
        }
        __syncthreads();  // relu(z2) read before dz1 takes its place
#pragma unroll
        for (int v = 0; v < 16; ++v) {
            const int j = 8 * (v / 4) + 4 * (int)half + (v % 4);
            s_r[col * LD + j] = w1[j] * x + b1[j] > 0.f ? dh0[v] : 0.f;
            s_r[col * LD + 32 + j] = w1[32 + j] * x + b1[32 + j] > 0.f ? dh1[v] : 0.f;
        }
        __syncthreads();
        for (int sm = 0; sm < CH; ++sm) {
            const float dz1 = s_r[sm * LD + l];
            acc_w1 += dz1 * s_x[w][sm];
            acc_b1 += dz1;
        }
        __syncthreads();  // staging free for the next step
    }
    // wavefront partials: dW2 blocks as [k][j], then the vector sums
    float* s_gw = s_buf + w * HID * HID;
#pragma unroll
    for (int v = 0; v < 16; ++v) {
        const int k = 8 * (v / 4) + 4 * (int)half + (v % 4);
        s_gw[k * HID + col] = gw00[v];
        s_gw[k * HID + 32 + col] = gw01[v];
        s_gw[(32 + k) * HID + col] = gw10[v];
        s_gw[(32 + k) * HID + 32 + col] = gw11[v];
    }
#pragma unroll
    for (int dd = 32; dd >= 1; dd >>= 1) {
        acc_loss += __shfl_xor(acc_loss, dd, WAVE);
        acc_b3 += __shfl_xor(acc_b3, dd, WAVE);
    }
    s_vec[w][0][l] = acc_w3;
    s_vec[w][1][l] = acc_b2;
    s_vec[w][2][l] = acc_w1;
    s_vec[w][3][l] = acc_b1;
    if (l == 0) {
        s_vec[w][4][0] = acc_b3;
        s_vec[w][5][0] = acc_loss;
    }
    __syncthreads();
    // chain rule through the weight parametrisation, then this block's sums
    float* out = partial + (size_t)blockIdx.x * (NPARAM + 1);
    for (int i = tid; i < HID * HID; i += MLP_T) {
        float t = 0.f;
#pragma unroll
        for (int ww = 0; ww < NWV; ++ww) t += s_buf[ww * HID * HID + i];
        out[O_V2 + i] = t * deff<MONO>(params[O_V2 + i]);
    }
    if (tid < HID) {
        float v[4] = {0.f, 0.f, 0.f, 0.f};
#pragma unroll
        for (int ww = 0; ww < NWV; ++ww)
#pragma unroll
            for (int q = 0; q < 4; ++q) v[q] += s_vec[ww][q][tid];
        out[O_V3 + tid] = v[0] * deff<MONO>(params[O_V3 + tid]);
        out[O_B2 + tid] = v[1];
        out[O_V1 + tid] = v[2] * deff<MONO>(params[O_V1 + tid]);
        out[O_B1 + tid] = v[3];
    }
    if (tid == 0) {
        float t3 = 0.f, tl = 0.f;
        for (int ww = 0; ww < NWV; ++ww) {
            t3 += s_vec[ww][4][0];
            tl += s_vec[ww][5][0];
        }
        out[O_B3] = t3;
        out[NPARAM] = tl;
    }
}

// Sum of the per-block gradients (and loss) into grad[NPARAM + 1].
__global__ void k_mlp_reduce(const float* __restrict__ partial, uint32_t blocks,
                             float* __restrict__ grad) {
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i > NPARAM) return;
    float s = 0.f;
    for (uint32_t b = 0; b < blocks; ++b) s += partial[(size_t)b * (NPARAM + 1) + i];
    grad[i] = s;
}

// Adam (Kingma & Ba 2015) on every parameter; loss_acc collects the epoch's
// loss sum.
__global__ void k_adam(float* __restrict__ params, float* __restrict__ m, float* __restrict__ v,
                       const float* __restrict__ grad, float lr, float b1, float b2, float eps,
                       float c1, float c2, float* __restrict__ loss_acc) {
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i == 0) *loss_acc += grad[NPARAM];
    if (i >= NPARAM) return;
    const float g = grad[i];
    const float mi = b1 * m[i] + (1.f - b1) * g;
    const float vi = b2 * v[i] + (1.f - b2) * g * g;
    m[i] = mi;
    v[i] = vi;
    params[i] -= lr * (mi / c1) / (sqrtf(vi / c2) + eps);
}

// ------------------------------------------------------------------ LUT
// F(W) = (dense sample keys in cells < W + rest * f(W / 2^24)) / S, in 0.32
// fixed point, for every cell start W in [0, 2^24]; f = the network clamped
// to [0, 1] (KIND 0), x (KIND 1, equal-width cells) or 0 (KIND 2).
enum { LUT_NET = 0, LUT_IDENTITY = 1, LUT_ZERO = 2 };

__device__ __forceinline__ uint32_t dense_before(const uint32_t* __restrict__ dense,
                                                 const uint32_t* __restrict__ dense_cum,
                                                 uint32_t nd, uint32_t w) {
    uint32_t a = 0, z = nd;  // dense cells < w
    while (a < z) {
        const uint32_t mid = (a + z) >> 1;
        if (dense[mid] < w) a = mid + 1; else z = mid;
    }
    return dense_cum[a];
}

// The cells without a network: f = x (equal-width cells) or 0.
template <int KIND>
__global__ __launch_bounds__(256) void k_lut_eval(const LearnedHeader* __restrict__ hdr,
                                                  const uint32_t* __restrict__ dense,
                                                  const uint32_t* __restrict__ dense_cum,
                                                  uint32_t* __restrict__ lut) {
    const uint32_t nd = hdr->dense, S = hdr->sample;
    const double rest = (double)(S - hdr->dense_keys), invS = 1.0 / (double)S;
    for (uint32_t c = blockIdx.x * 256 + threadIdx.x; c <= LUT_CELLS; c += gridDim.x * 256) {
        const float x = (float)c * (1.f / (float)LUT_CELLS);
        const float f = KIND == LUT_IDENTITY ? x : 0.f;
        const double F = ((double)dense_before(dense, dense_cum, nd, c) + rest * (double)f) * invS;
        uint32_t q = (uint32_t)fmin(F * 4294967295.0, 4294967295.0);
        if (c == 0) q = 0;
        if (c == LUT_CELLS) q = 0xFFFFFFFFu;
        lut[c] = q;
    }
}

// The network's LUT entries on the matrix cores (the 64 x 64 layer is a dense
// contraction over all 2^24 + 1 cells).  Each wavefront takes 32 cells at a
// time and forms z2^T = W2 h1^T as two 32 x 32 blocks (hidden units 0-31 and
// 32-63) with K = 64 in 32 steps of v_mfma_f32_32x32x2f32.  In step s lane l
// supplies W2[32t + l % 32][2s + l / 32] (the A operands of both blocks, held
// in registers for the whole kernel) and h1 of its cell c = base + l % 32 at
// hidden unit 2s + l / 32 (the B operand, computed in place), and receives
// z2 of its cell at units 32t + 8(v / 4) + 4(l / 32) + v % 4 in accumulator
// register v.  The output layer sums those, the two lanes of a cell (l and
// l + 32) add their halves, and the first 32 lanes write the cells.  The sums
// run in another order than the scalar form's, within the same fp32 error
// bound.
template <bool MONO>
__global__ __launch_bounds__(256) void k_lut_net(const float* __restrict__ params,
                                                 const LearnedHeader* __restrict__ hdr,
                                                 const uint32_t* __restrict__ dense,
                                                 const uint32_t* __restrict__ dense_cum,
                                                 uint32_t* __restrict__ lut) {
    __shared__ float s_b2[HID], s_w3[HID];
    const uint32_t l = lane_id(), half = l / 32, col = l % 32;
    if (threadIdx.x < HID) {
        s_b2[threadIdx.x] = params[O_B2 + threadIdx.x];
        s_w3[threadIdx.x] = eff<MONO>(params[O_V3 + threadIdx.x]);
    }
    float a0[HID / 2], a1[HID / 2], w1v[HID / 2], b1v[HID / 2];
#pragma unroll
    for (int st = 0; st < HID / 2; ++st) {
        const int j = 2 * st + (int)half;
        a0[st] = eff<MONO>(params[O_V2 + (int)col * HID + j]);
        a1[st] = eff<MONO>(params[O_V2 + (32 + (int)col) * HID + j]);
        w1v[st] = eff<MONO>(params[O_V1 + j]);
        b1v[st] = params[O_B1 + j];
    }
    __syncthreads();
    const float b3 = params[O_B3];
    const uint32_t nd = hdr->dense, S = hdr->sample;
    const double rest = (double)(S - hdr->dense_keys), invS = 1.0 / (double)S;
    const uint32_t wv = blockIdx.x * (256 / WAVE) + threadIdx.x / WAVE, nwv = gridDim.x * (256 / WAVE);
    for (uint32_t base = wv * 32; base <= LUT_CELLS; base += nwv * 32) {  // uniform per wavefront
        const uint32_t c = base + col;
        const float x = (float)c * (1.f / (float)LUT_CELLS);
        f32x16 z0 = {}, z1 = {};
#pragma unroll
        for (int st = 0; st < HID / 2; ++st) {
            const float h = fmaxf(w1v[st] * x + b1v[st], 0.f);
            z0 = __builtin_amdgcn_mfma_f32_32x32x2f32(a0[st], h, z0, 0, 0, 0);
            z1 = __builtin_amdgcn_mfma_f32_32x32x2f32(a1[st], h, z1, 0, 0, 0);
        }
        float part = 0.f;
#pragma unroll
        for (int v = 0; v < 16; ++v) {
            const int k = 8 * (v / 4) + 4 * (int)half + (v % 4);
            part += s_w3[k] * fmaxf(z0[v] + s_b2[k], 0.f);
            part += s_w3[32 + k] * fmaxf(z1[v] + s_b2[32 + k], 0.f);
        }
        const float out = b3 + (part + __shfl_xor(part, 32, WAVE));
        if (half == 0 && c <= LUT_CELLS) {
            const float f = fminf(fmaxf(out, 0.f), 1.f);
            const double F = ((double)dense_before(dense, dense_cum, nd, c) + rest * (double)f) * invS;
            uint32_t q = (uint32_t)fmin(F * 4294967295.0, 4294967295.0);
            if (c == 0) q = 0;
            if (c == LUT_CELLS) q = 0xFFFFFFFFu;
            lut[c] = q;
        }
    }
}

// Running maximum over the 2^24 + 1 LUT entries: per-tile scan, scan of the
// tile maxima (one workgroup), then each tile applies its carry.
constexpr int LUT_TILE = 4096;
__device__ __forceinline__ uint32_t wave_inclusive_max(uint32_t v) {
    const uint32_t lane = lane_id();
#pragma unroll
    for (int d = 1; d < WAVE; d <<= 1) {
        const uint32_t t = __shfl_up(v, d, WAVE);
        if (lane >= (uint32_t)d) v = max(v, t);
    }
    return v;
}
__global__ __launch_bounds__(256) void k_lut_tilemax(const uint32_t* __restrict__ lut, uint32_t n,
                                                     uint32_t* __restrict__ tmax) {
    __shared__ uint32_t s[NWAVES];
    const uint32_t t0 = blockIdx.x * LUT_TILE;
    uint32_t m = 0;
    for (uint32_t i = t0 + threadIdx.x; i < min(n, t0 + LUT_TILE); i += 256) m = max(m, lut[i]);
#pragma unroll
    for (int d = 32; d >= 1; d >>= 1) m = max(m, (uint32_t)__shfl_xor(m, d, WAVE));
    if (lane_id() == 0) s[threadIdx.x / WAVE] = m;
    __syncthreads();
    if (threadIdx.x == 0) tmax[blockIdx.x] = max(max(s[0], s[1]), max(s[2], s[3]));
}
__global__ __launch_bounds__(256) void k_lut_carry(uint32_t* tmax, uint32_t tiles) {
    // exclusive running max of the tile maxima (one workgroup)
    __shared__ uint32_t s[NWAVES];
    uint32_t carry = 0;
    for (uint32_t b = 0; b < tiles; b += 256) {
        const uint32_t i = b + threadIdx.x;
        const uint32_t v = i < tiles ? tmax[i] : 0u;
        const uint32_t inc = wave_inclusive_max(v);
        if (lane_id() == WAVE - 1) s[threadIdx.x / WAVE] = inc;
        __syncthreads();
        uint32_t before = carry, all = carry;
        for (int w = 0; w < NWAVES; ++w) {
            if (w < (int)(threadIdx.x / WAVE)) before = max(before, s[w]);
            all = max(all, s[w]);
        }
        const uint32_t excl = max(before, __shfl_up(inc, 1, WAVE) * (lane_id() > 0 ? 1u : 0u));
        __syncthreads();
        if (i < tiles) tmax[i] = excl;
        carry = all;
    }
}
__global__ __launch_bounds__(256) void k_lut_apply(uint32_t* __restrict__ lut, uint32_t n,
                                                   const uint32_t* __restrict__ tcarry) {
    __shared__ uint32_t s[NWAVES];
    const uint32_t t0 = blockIdx.x * LUT_TILE;
    uint32_t carry = tcarry[blockIdx.x];
    // 16 consecutive entries per thread, scanned in place
    const uint32_t i0 = t0 + threadIdx.x * 16;
    uint32_t v[16], m = 0;
#pragma unroll
    for (int k = 0; k < 16; ++k) {
        v[k] = i0 + k < n ? lut[i0 + k] : 0u;
        m = max(m, v[k]);
        v[k] = m;
    }
    const uint32_t inc = wave_inclusive_max(m);
    if (lane_id() == WAVE - 1) s[threadIdx.x / WAVE] = inc;
    __syncthreads();
    uint32_t before = carry;
    for (int w = 0; w < (int)(threadIdx.x / WAVE); ++w) before = max(before, s[w]);
    uint32_t prev = __shfl_up(inc, 1, WAVE);
    if (lane_id() == 0) prev = 0;
    before = max(before, prev);
#pragma unroll
    for (int k = 0; k < 16; ++k)
        if (i0 + k < n) lut[i0 + k] = max(before, v[k]);
}

// ------------------------------------------------------------------ buckets
__device__ __forceinline__ uint32_t bucket_of_lut(uint32_t q, uint32_t B) {
    return (uint32_t)(((uint64_t)q * B) >> 32);
}

// Splitters of every cell that owns two or more buckets: for cell W with
// buckets [b0, b1) and sample keys sample[s_lo, s_hi) (sorted), splitter i
// (1 <= i < b1 - b0) is sample[s_lo + i * m / (b1 - b0)], stored at
// splitters[b0 + i - 1]; a cell with no sample keys gets +inf splitters.
__global__ __launch_bounds__(256) void k_splitters(const uint32_t* __restrict__ lut,
                                                   const uint64_t* __restrict__ sample,
                                                   uint32_t S, LearnedHeader* hdr,
                                                   uint64_t* __restrict__ splitters) {
    const uint64_t lo = hdr->lo, hi = hdr->hi;
    const uint32_t cp = hdr->cp, B = hdr->buckets;
    uint32_t heavy = 0;
    for (uint32_t w = blockIdx.x * 256 + threadIdx.x; w < LUT_CELLS; w += gridDim.x * 256) {
        const uint32_t b0 = bucket_of_lut(lut[w], B), b1 = bucket_of_lut(lut[w + 1], B);
        if (b1 < b0 + 2) continue;
        ++heavy;
        // sample range of cell w (windows of the sorted sample never decrease)
        uint32_t a = 0, z = S;
        while (a < z) {
            const uint32_t mid = (a + z) >> 1;
            if (window_of(sample[mid], lo, hi, cp) < w) a = mid + 1; else z = mid;
        }
        const uint32_t s_lo = a;
        z = S;
        while (a < z) {
            const uint32_t mid = (a + z) >> 1;
            if (window_of(sample[mid], lo, hi, cp) <= w) a = mid + 1; else z = mid;
        }
        const uint32_t m = a - s_lo, k = b1 - b0;
        for (uint32_t i = 1; i < k; ++i)
            splitters[b0 + i - 1] = m ? sample[s_lo + (uint32_t)(((uint64_t)i * m) / k)] : ~0ull;
    }
    if (heavy) atomicAdd(&hdr->heavy, heavy);
}

// Sub-cells of a heavy cell.  Its k - 1 splitters share their top P bits (P =
// common prefix of the first and the last); a key whose top P bits are below
// (above) that prefix counts 0 (k - 1) splitters.  Otherwise its next s bits,
// s = min(16, 64 - P, ceil(log2 k) + 3), index a table of 2^s entries:
// entry v = the splitters below the first code with those bits equal to v,
// so the key only searches the splitters of its own sub-cell -- with about
// eight sub-cells per bucket, mostly none or one.  The cell's slot at
// subtab[16 b0 ..] holds a 16-byte header {u16 P, u16 s, u32 0, u64 prefix}
// and the 2^s entries (2^s + 8 <= 16k: slots never overlap, since cells own
// disjoint bucket ranges).
__device__ __forceinline__ uint32_t sub_bits_for(uint32_t k, uint32_t P) {
    const uint32_t lg = 32u - (uint32_t)__clz(k - 1u);  // ceil(log2 k), k >= 2
    return min(64u - P, min(16u, lg + 3u));
}

// Per-cell info for the sort (see bucket.h): buckets of every cell and, for
// heavy cells, the sub-cell key when the splitters' prefix extends at most
// INLINE_PREFIX_BITS below the cell.
__global__ __launch_bounds__(256) void k_cellinfo(const uint32_t* __restrict__ lut,
                                                  const LearnedHeader* __restrict__ hdr,
                                                  const uint64_t* __restrict__ splitters,
                                                  uint64_t* __restrict__ info) {
    const uint32_t B = hdr->buckets, cp = hdr->cp;
    for (uint32_t w = blockIdx.x * 256 + threadIdx.x; w < LUT_CELLS; w += gridDim.x * 256) {
        const uint32_t b0 = bucket_of_lut(lut[w], B), b1 = bucket_of_lut(lut[w + 1], B);
        uint64_t v = (uint64_t)b0 | ((uint64_t)b1 << 16);
        if (b1 >= b0 + 2) {
            const uint32_t k = b1 - b0;
            const uint64_t first = splitters[b0], last = splitters[b0 + k - 2];
            const uint32_t P = first == last ? 64u : (uint32_t)__clzll((long long)(first ^ last));
            const uint32_t s = sub_bits_for(k, P);
            const uint32_t below = cp + 24;  // bits of prefix and cell
            if (P < 64 && below < 64 && P >= below && P - below <= (uint32_t)INLINE_PREFIX_BITS) {
                const uint32_t e = P - below;
                const uint64_t extra = e ? (first << below) >> (64 - e) : 0ull;
                v |= ((uint64_t)P << 32) | ((uint64_t)s << 39) | (extra << 44);
            } else {
                v |= 1ull << 63;
            }
        }
        info[w] = v;
    }
}

// One thread per slot e of subtab: the cell owning bucket e / SUB_SLOT (the
// last cell whose first bucket is <= that bucket), then its header or entry.
__global__ __launch_bounds__(256) void k_subtables(const uint32_t* __restrict__ lut,
                                                   const LearnedHeader* __restrict__ hdr,
                                                   const uint64_t* __restrict__ splitters,
                                                   uint16_t* __restrict__ subtab) {
    const uint32_t B = hdr->buckets;
    for (uint32_t e = blockIdx.x * 256 + threadIdx.x; e < SUB_SLOT * B; e += gridDim.x * 256) {
        const uint32_t bk = e / SUB_SLOT;
        uint32_t a = 0, z = LUT_CELLS;  // first cell whose first bucket is > bk
        while (a < z) {
            const uint32_t mid = (a + z) >> 1;
            if (bucket_of_lut(lut[mid], B) <= bk) a = mid + 1; else z = mid;
        }
        if (a == 0) continue;
        const uint32_t W = a - 1;
        const uint32_t b0 = bucket_of_lut(lut[W], B), b1 = bucket_of_lut(lut[W + 1], B);
        if (b1 < b0 + 2 || bk >= b1) continue;
        const uint32_t k = b1 - b0;
        const uint64_t first = splitters[b0], last = splitters[b0 + k - 2];
        const uint32_t P = first == last ? 64u : (uint32_t)__clzll((long long)(first ^ last));
        const uint32_t s = sub_bits_for(k, P);
        const uint64_t prefix = P >= 64 ? first : (P ? first & ~(~0ull >> P) : 0ull);
        const uint32_t local = e - SUB_SLOT * b0;
        if (local < 8) {
            uint32_t v = 0;
            if (local == 0) v = P;
            else if (local == 1) v = s;
            else if (local >= 4) v = (uint32_t)(prefix >> (16 * (local - 4))) & 0xFFFFu;
            subtab[e] = (uint16_t)v;
            continue;
        }
        const uint32_t v = local - 8;
        if (v >= (1u << s)) continue;
        const uint64_t start = prefix | ((uint64_t)v << (64 - P - s));
        uint32_t x = 0, y = k - 1;  // splitters < start
        while (x < y) {
            const uint32_t mid = (x + y) >> 1;
            if (splitters[b0 + mid] < start) x = mid + 1; else y = mid;
        }
        subtab[e] = (uint16_t)x;
    }
}

// ------------------------------------------------------------------ bucket passes
// Two stable LSD passes over the 16-bit ids (low byte, then high byte) on
// the whole array as one segment; the same tile / group / segment scans as
// radix.hip.  The pass moves (code, index, id) through LDS one array at a
// time.
template <int ITEMS>
__global__ __launch_bounds__(BLOCK) void k_bcount(const uint16_t* __restrict__ bid, uint32_t n,
                                                  int shift, uint32_t* __restrict__ cnt) {
    constexpr uint32_t TILE = BLOCK * ITEMS;
    __shared__ uint32_t s_h[HIST_WORDS];
    const uint32_t t = xcd_remap(blockIdx.x, gridDim.x), w = threadIdx.x / WAVE, lane = lane_id();
    const uint32_t base = t * TILE;
    if (base >= n) return;
    const uint32_t nvalid = min(TILE, n - base);
    uint32_t b[ITEMS];
#pragma unroll
    for (int i = 0; i < ITEMS; ++i) {
        const uint32_t p = w * WAVE * ITEMS + i * WAVE + lane;
        b[i] = p < nvalid ? (uint32_t)bid[base + p] : 0u;
    }
    tile_histogram<ITEMS>([&](int i) { return (b[i] >> shift) & 255u; }, nvalid, s_h,
                          cnt + (size_t)t * 256);
}

template <int ITEMS, bool CARRY>
__global__ __launch_bounds__(BLOCK) void k_bscatter(const uint64_t* __restrict__ ksrc,
                                                    const uint32_t* __restrict__ vsrc,
                                                    const uint16_t* __restrict__ bsrc,
                                                    const uint64_t* __restrict__ k0src,
                                                    uint64_t* __restrict__ kdst,
                                                    uint32_t* __restrict__ vdst,
                                                    uint16_t* __restrict__ bdst,
                                                    uint64_t* __restrict__ k0dst, uint32_t n,
                                                    int shift, const uint32_t* __restrict__ cnt,
                                                    const uint32_t* __restrict__ gtot,
                                                    const uint32_t* __restrict__ binstart) {
    constexpr uint32_t TILE = BLOCK * ITEMS;
    __shared__ uint64_t s_buf[TILE];
    __shared__ uint16_t s_bid[TILE];
    __shared__ uint32_t s_whist[NWAVES * 256];
    __shared__ uint32_t s_binstart[256];
    __shared__ uint32_t s_gbase[256];
    __shared__ uint32_t s_scan[NWAVES];
    const uint32_t t = xcd_remap(blockIdx.x, gridDim.x), tid = threadIdx.x, w = tid / WAVE,
                   lane = lane_id();
    const uint32_t base = t * TILE;
    if (base >= n) return;
    const uint32_t nvalid = min(TILE, n - base);
    // all three arrays are loaded before the ranking so that their loads overlap
    uint64_t kv[ITEMS], k0v[ITEMS];
    uint32_t vv[ITEMS], bv[ITEMS], dig[ITEMS];
#pragma unroll
    for (int i = 0; i < ITEMS; ++i) {
        const uint32_t p = w * WAVE * ITEMS + i * WAVE + lane;
        const bool ok = p < nvalid;
        bv[i] = ok ? bsrc[base + p] : 0xFFFFu;
        kv[i] = ok ? ksrc[base + p] : 0ull;
        if (CARRY) k0v[i] = ok ? k0src[base + p] : 0ull;
        vv[i] = vsrc ? (ok ? vsrc[base + p] : 0u) : base + p;  // no source: input order
        dig[i] = (bv[i] >> shift) & 255u;
    }
    uint32_t pos[ITEMS], bc = 0;
    rank_digits<8, ITEMS>(dig, nvalid, pos, s_whist, s_binstart, s_scan, &bc);
    if (tid < 256) {
        const uint32_t g = t / GROUP_TILES;
        s_gbase[tid] = binstart[tid] + gtot[(size_t)g * 256 + tid] + cnt[(size_t)t * 256 + tid] -
                       s_binstart[tid];
    }
#pragma unroll
    for (int i = 0; i < ITEMS; ++i) {
        s_buf[pos[i]] = kv[i];
        s_bid[pos[i]] = (uint16_t)bv[i];
    }
    __syncthreads();
    // codes and ids leave in digit order: neighbouring lanes write neighbouring
    // addresses inside each digit's run
    uint32_t dst[ITEMS];
#pragma unroll
    for (int i = 0; i < ITEMS; ++i) {
        const uint32_t p = i * BLOCK + tid;
        dst[i] = 0;
        if (p < nvalid) {
            const uint32_t bb = s_bid[p];
            dst[i] = s_gbase[(bb >> shift) & 255u] + p;
            kdst[dst[i]] = s_buf[p];
            if (bdst) bdst[dst[i]] = (uint16_t)bb;
        }
    }
    __syncthreads();
    if (CARRY) {  // the first refinement key travels like the code
#pragma unroll
        for (int i = 0; i < ITEMS; ++i) s_buf[pos[i]] = k0v[i];
        __syncthreads();
#pragma unroll
        for (int i = 0; i < ITEMS; ++i) {
            const uint32_t p = i * BLOCK + tid;
            if (p < nvalid) k0dst[dst[i]] = s_buf[p];
        }
        __syncthreads();
    }
    uint32_t* s_v = (uint32_t*)s_buf;
#pragma unroll
    for (int i = 0; i < ITEMS; ++i) s_v[pos[i]] = vv[i];
    __syncthreads();
#pragma unroll
    for (int i = 0; i < ITEMS; ++i) {
        const uint32_t p = i * BLOCK + tid;
        if (p < nvalid) vdst[dst[i]] = s_v[p];
    }
}

// seg[b] = first position whose id is >= b, for b in [0, B]; ids sorted.
__global__ __launch_bounds__(256) void k_bucket_bounds(const uint16_t* __restrict__ bid, uint32_t n,
                                                       uint32_t B, uint64_t* __restrict__ seg) {
    // thread c takes positions [8c, 8c + 8) of 0..n (one 16-byte load of ids
    // when the array is 16-byte aligned and the chunk lies inside it)
    const bool vec = ((uintptr_t)bid & 15u) == 0;
    for (uint64_t c = blockIdx.x * 256ull + threadIdx.x; c * 8 <= n; c += gridDim.x * 256ull) {
        const uint32_t i0 = (uint32_t)(c * 8);
        uint32_t id[8];
        if (vec && i0 + 8 <= n) {
            const uint4 q = *reinterpret_cast<const uint4*>(bid + i0);
            const uint32_t w[4] = {q.x, q.y, q.z, q.w};
#pragma unroll
            for (int j = 0; j < 4; ++j) {
                id[2 * j] = w[j] & 0xFFFFu;
                id[2 * j + 1] = w[j] >> 16;
            }
        } else {
#pragma unroll
            for (int j = 0; j < 8; ++j) id[j] = i0 + j < n ? (uint32_t)bid[i0 + j] : B;
        }
        // buckets prev..cur start at position i: prev = 1 + the id before i
        // (0 at i = 0), cur = the id at i (B at i = n)
        uint32_t prev = i0 == 0 ? 0u : (uint32_t)bid[i0 - 1] + 1u;
#pragma unroll
        for (int j = 0; j < 8; ++j) {
            const uint32_t i = i0 + j;
            if (i > n) break;
            const uint32_t cur = i == n ? B : id[j];
            for (uint32_t b = prev; b <= cur && b <= B; ++b) seg[b] = i;
            prev = cur + 1u;
        }
    }
}

// Exclusive scan of the tile counts within groups of GROUP_TILES tiles (in
// place) and the group totals, for the whole array as one segment.
__global__ __launch_bounds__(256) void k_lgroup_scan(uint32_t* __restrict__ cnt, uint32_t tiles,
                                                     uint32_t* __restrict__ gtot) {
    const uint32_t g = blockIdx.x, d = threadIdx.x;
    const uint32_t t0 = g * GROUP_TILES, nt = min((uint32_t)GROUP_TILES, tiles - t0);
    uint32_t v[GROUP_TILES];
#pragma unroll
    for (int i = 0; i < GROUP_TILES; ++i) v[i] = (uint32_t)i < nt ? cnt[(size_t)(t0 + i) * 256 + d] : 0u;
    uint32_t run = 0;
#pragma unroll
    for (int i = 0; i < GROUP_TILES; ++i) {
        if ((uint32_t)i < nt) cnt[(size_t)(t0 + i) * 256 + d] = run;
        run += v[i];
    }
    gtot[(size_t)g * 256 + d] = run;
}
// Scan of the group totals (in place) and the digit starts (one workgroup).
__global__ __launch_bounds__(256) void k_lseg_scan(uint32_t* __restrict__ gtot, uint32_t groups,
                                                   uint32_t* __restrict__ binstart) {
    __shared__ uint32_t scratch[NWAVES];
    const uint32_t d = threadIdx.x;
    uint32_t run = 0;
    constexpr int U = 64;  // group totals in flight per thread
    for (uint32_t g0 = 0; g0 < groups; g0 += U) {
        uint32_t v[U];
#pragma unroll
        for (int i = 0; i < U; ++i) v[i] = g0 + i < groups ? gtot[(size_t)(g0 + i) * 256 + d] : 0u;
#pragma unroll
        for (int i = 0; i < U; ++i) {
            if (g0 + i < groups) gtot[(size_t)(g0 + i) * 256 + d] = run;
            run += v[i];
        }
    }
    uint32_t tot;
    binstart[d] = block_exclusive_sum(run, scratch, &tot);
}

// Seeded sample: string index splitmix64(seed + golden * (j + 1)) mod n for
// j < S, drawn with replacement.
__global__ void k_sample_idx(uint32_t* __restrict__ sel, uint32_t S, uint32_t n, uint64_t seed) {
    for (uint32_t j = blockIdx.x * 256 + threadIdx.x; j < S; j += gridDim.x * 256)
        sel[j] = (uint32_t)(splitmix64(seed + 0x9E3779B97F4A7C15ull * ((uint64_t)j + 1)) % n);
}

// Header from the sorted sample: extremes and their common prefix.
__global__ void k_learned_header(const uint64_t* __restrict__ sample, uint32_t S,
                                 LearnedHeader* hdr, uint32_t mode, uint32_t flags) {
    const uint64_t lo = sample[0], hi = sample[S - 1];
    hdr->lo = lo;
    hdr->hi = hi;
    hdr->cp = lo == hi ? 64u : (uint32_t)__clzll((long long)(lo ^ hi));
    hdr->buckets = LEARNED_BUCKETS;
    hdr->mode = mode;
    hdr->sample = S;
    hdr->steps = 0;
    hdr->last_loss = 0.f;
    hdr->heavy = 0;
    hdr->dense = 0;
    hdr->dense_keys = 0;
    hdr->trained = 0;
    hdr->flags = flags;
}

// Dense-cell flags of every sample position j (sorted sample): bit 0 = its
// cell holds at least two buckets' worth of sample keys (count * B >= 2 S)
// and at least DENSE_MIN of them (fewer is sampling noise, not a spike),
// bit 1 = j is the first sample key of such a cell.  The cell's sample range
// comes from two binary searches (windows of the sorted sample never
// decrease).
__global__ __launch_bounds__(256) void k_dense_flags(const uint64_t* __restrict__ sample, uint32_t S,
                                                     const LearnedHeader* __restrict__ hdr,
                                                     uint32_t use_dense, uint8_t* __restrict__ flags) {
    const uint64_t lo = hdr->lo, hi = hdr->hi;
    const uint32_t cp = hdr->cp;
    for (uint32_t j = blockIdx.x * 256 + threadIdx.x; j < S; j += gridDim.x * 256) {
        uint8_t f = 0;
        if (use_dense) {
            const uint32_t w = window_of(sample[j], lo, hi, cp);
            uint32_t a = 0, z = j;
            while (a < z) {
                const uint32_t mid = (a + z) >> 1;
                if (window_of(sample[mid], lo, hi, cp) < w) a = mid + 1; else z = mid;
            }
            const uint32_t first = a;
            a = j + 1;
            z = S;
            while (a < z) {
                const uint32_t mid = (a + z) >> 1;
                if (window_of(sample[mid], lo, hi, cp) <= w) a = mid + 1; else z = mid;
            }
            const uint64_t cnt = a - first;
            if (cnt * LEARNED_BUCKETS >= 2ull * S && cnt >= DENSE_MIN)
                f = (uint8_t)(1u | (j == first ? 2u : 0u));
        }
        flags[j] = f;
    }
}

// Two counters per position scanned over the sample in tiles of SCAN_TILE:
// dense keys before j, and dense cells started before j.
constexpr uint32_t SCAN_TILE = 4096;
__global__ __launch_bounds__(256) void k_flag_sums(const uint8_t* __restrict__ flags, uint32_t S,
                                                   uint2* __restrict__ tsum) {
    __shared__ uint32_t s0[NWAVES], s1[NWAVES];
    const uint32_t t0 = blockIdx.x * SCAN_TILE;
    uint32_t a = 0, b = 0;
    for (uint32_t i = t0 + threadIdx.x; i < min(S, t0 + SCAN_TILE); i += 256) {
        a += flags[i] & 1u;
        b += (flags[i] >> 1) & 1u;
    }
#pragma unroll
    for (int d = 32; d >= 1; d >>= 1) {
        a += __shfl_xor(a, d, WAVE);
        b += __shfl_xor(b, d, WAVE);
    }
    if (lane_id() == 0) {
        s0[threadIdx.x / WAVE] = a;
        s1[threadIdx.x / WAVE] = b;
    }
    __syncthreads();
    if (threadIdx.x == 0) tsum[blockIdx.x] = make_uint2(s0[0] + s0[1] + s0[2] + s0[3], s1[0] + s1[1] + s1[2] + s1[3]);
}
// Exclusive scan of the tile sums (one workgroup); totals into the header.
__global__ __launch_bounds__(256) void k_flag_scan(uint2* __restrict__ tsum, uint32_t tiles,
                                                   LearnedHeader* hdr) {
    __shared__ uint32_t sc0[NWAVES], sc1[NWAVES];
    uint32_t c0 = 0, c1 = 0;
    for (uint32_t b = 0; b < tiles; b += 256) {
        const uint32_t i = b + threadIdx.x;
        const uint2 v = i < tiles ? tsum[i] : make_uint2(0u, 0u);
        uint32_t t0, t1;
        const uint32_t e0 = block_exclusive_sum(v.x, sc0, &t0);
        const uint32_t e1 = block_exclusive_sum(v.y, sc1, &t1);
        if (i < tiles) tsum[i] = make_uint2(c0 + e0, c1 + e1);
        c0 += t0;
        c1 += t1;
    }
    if (threadIdx.x == 0) {
        hdr->dense_keys = c0;
        hdr->dense = c1;
    }
}
// Per tile: positions of every sample key among the dense / other keys; the
// other keys become training pairs x = W / 2^24, y = (rank + 0.5) / count,
// written compactly; each dense cell's first key records the cell and the
// dense keys before it.
__global__ __launch_bounds__(256) void k_flag_apply(const uint8_t* __restrict__ flags,
                                                    const uint64_t* __restrict__ sample, uint32_t S,
                                                    const uint2* __restrict__ tsum,
                                                    const LearnedHeader* __restrict__ hdr,
                                                    float* __restrict__ x, float* __restrict__ y,
                                                    uint32_t* __restrict__ dense,
                                                    uint32_t* __restrict__ dense_cum) {
    __shared__ uint32_t sc0[NWAVES], sc1[NWAVES];
    const uint64_t lo = hdr->lo, hi = hdr->hi;
    const uint32_t cp = hdr->cp, nd = hdr->dense, dk = hdr->dense_keys;
    const uint32_t rest = S - dk;
    const float inv_rest = rest ? 1.f / (float)rest : 0.f;
    const uint32_t t0 = blockIdx.x * SCAN_TILE;
    uint2 run = tsum[blockIdx.x];
    for (uint32_t b = t0; b < min(S, t0 + SCAN_TILE); b += 256) {
        const uint32_t j = b + threadIdx.x;
        const uint32_t f = j < S ? flags[j] : 0u;
        uint32_t t_a, t_b;
        const uint32_t e0 = block_exclusive_sum(f & 1u, sc0, &t_a);
        const uint32_t e1 = block_exclusive_sum((f >> 1) & 1u, sc1, &t_b);
        if (j < S) {
            const uint32_t before_dense = run.x + e0;
            const uint32_t w = window_of(sample[j], lo, hi, cp);
            if (f & 1u) {
                if (f & 2u) {
                    dense[run.y + e1] = w;
                    dense_cum[run.y + e1] = before_dense;
                }
            } else {
                const uint32_t r = j - before_dense;
                x[r] = (float)w * (1.f / (float)LUT_CELLS);
                y[r] = ((float)r + 0.5f) * inv_rest;
            }
        }
        run.x += t_a;
        run.y += t_b;
    }
    if (blockIdx.x == 0 && threadIdx.x == 0) dense_cum[nd] = dk;
}

__global__ void k_learned_finish(LearnedHeader* hdr, const float* __restrict__ loss_acc,
                                 uint32_t steps, uint32_t trained) {
    hdr->steps = steps;
    hdr->trained = trained;
    hdr->last_loss = trained ? *loss_acc / (float)trained : 0.f;
}

// Buckets larger than the LDS sort's capacity go to the multi-tile radix
// passes (overflow): their number and their keys; each one joins the list the
// radix passes sort and the list of segments Step 3's run detection scans.
// Every other bucket of two or more keys joins the list of its LDS size
// class (<= 3,072, <= 4,096, <= 6,144, <= 8,192 keys); one atomic per
// wavefront and list.
__device__ __forceinline__ void wave_append(bool mine, const RunItem& it, RunItem* list,
                                            uint32_t* count) {
    const uint64_t m = ballot(mine);
    if (!m) return;
    const uint32_t lane = lane_id(), leader = (uint32_t)__ffsll((unsigned long long)m) - 1u;
    uint32_t base = 0;
    if (lane == leader) base = atomicAdd(count, (uint32_t)__popcll(m));
    base = readlane(base, (int)leader);
    if (mine) list[base + mbcnt(m)] = it;
}

__global__ __launch_bounds__(256) void k_bucket_classes(const uint64_t* __restrict__ seg, uint32_t B,
                                                        uint32_t* __restrict__ out,
                                                        RunItem* __restrict__ big_list,
                                                        uint32_t* __restrict__ big_count,
                                                        RunItem* __restrict__ scan_list,
                                                        uint32_t* __restrict__ scan_count,
                                                        RunItem* l0, RunItem* l1, RunItem* l2,
                                                        RunItem* l3, uint32_t* __restrict__ class_count) {
    uint32_t nb = 0, nk = 0;
    const uint32_t c1 = BLOCK * 12u, c2 = BLOCK * 16u, c3 = 2 * BLOCK * 12u;
    for (uint32_t b0 = blockIdx.x * 256; b0 < B; b0 += gridDim.x * 256) {  // uniform trip count
        const uint32_t b = b0 + threadIdx.x;
        uint32_t len = 0, st = 0;
        if (b < B) {
            st = (uint32_t)seg[b];
            len = (uint32_t)(seg[b + 1] - seg[b]);
        }
        const RunItem it{st, len, 0u, LCP_NONE};
        const bool big = len > LEARNED_LDS_CAP;
        if (big) {
            ++nb;
            nk += len;
        }
        wave_append(big, it, big_list, big_count);
        wave_append(big, it, scan_list, scan_count);
        const bool lds = len >= 2 && !big;
        wave_append(lds && len <= c1, it, l0, class_count + 0);
        wave_append(lds && len > c1 && len <= c2, it, l1, class_count + 1);
        wave_append(lds && len > c2 && len <= c3, it, l2, class_count + 2);
        wave_append(lds && len > c3, it, l3, class_count + 3);
    }
    if (nb) {
        atomicAdd(&out[0], nb);
        atomicAdd(&out[1], nk);
    }
}

// ------------------------------------------------------------------ per-bucket sort with the first refinement round
// One workgroup per bucket of 2..cap keys, in LDS:
//  1. sort (code, slot) by the code's varying digits (slot = position in the
//     bucket, which is input order);
//  2. run start of every position (the first position with the same code);
//  3. if some code repeats: sort (run start, first refinement key, slot) by
//     the key's varying digits, then by the run start's -- so every run of
//     equal codes is ordered by its first refinement key, ties by slot;
//  4. write the permutation (indices gathered by slot) and, in place of the
//     codes, a tie key per position: the first position of its group, where
//     a group is a run of equal (code, refinement key) whose key continues;
//     a bucket that still holds such a group joins the list of segments that
//     Step 3's run detection scans (with the larger buckets, whose codes are
//     left as they are).
// Every later refinement round proceeds as for any run.
// One size class of buckets: lmin < len <= lmax (and 2 <= len <= NW * 64 * ITEMS),
// one workgroup of NW wavefronts per bucket.
// Per item: its key and one word sr = slot | run start << 16 | the first
// refinement key continues << 31 (slot < 2^16, run start < 2^15).  Keys are
// sorted packed to their varying bits when that saves a digit pass.
template <int CODER, int ITEMS, int NW>
__global__ __launch_bounds__(NW * WAVE) void k_bucket_refine(uint64_t* __restrict__ codes,
                                                         uint32_t* __restrict__ perm,
                                                         const uint64_t* __restrict__ k0,
                                                         const RunItem* __restrict__ list,
                                                         const uint32_t* __restrict__ list_count,
                                                         int code_bits,
                                                         RunItem* __restrict__ scan_list,
                                                         uint32_t* __restrict__ scan_count) {
    constexpr uint32_t TILE = NW * WAVE * ITEMS;
    static_assert(TILE <= 32768, "slots fit 16 bits, run starts 15");
    __shared__ uint64_t s_k[TILE];
    __shared__ uint32_t s_sr[TILE];
    __shared__ uint32_t s_whist[NW * 256];
    __shared__ uint32_t s_binstart[256];
    __shared__ uint32_t s_scan[NW];
    __shared__ uint64_t s_or[NW], s_and[NW];
    uint32_t* s_k32 = reinterpret_cast<uint32_t*>(s_k);  // scratch while keys sit in registers
    const uint32_t nlist = *list_count;
    for (uint32_t it = blockIdx.x; it < nlist; it += gridDim.x) {
    const RunItem d = list[it];
    if (d.len < 2 || d.len > TILE) continue;  // never listed so; uniform per workgroup
    const uint32_t nvalid = d.len, start = d.start;
    const uint32_t w = threadIdx.x / WAVE, lane = lane_id();
    auto posof = [&](int i) { return w * WAVE * ITEMS + i * WAVE + lane; };
    // bits of 64-bit keys that vary over the valid items
    auto vary_of = [&](const uint64_t(&k)[ITEMS]) {
        uint64_t o = 0, a = ~0ull;
#pragma unroll
        for (int i = 0; i < ITEMS; ++i)
            if (posof(i) < nvalid) {
                o |= k[i];
                a &= k[i];
            }
#pragma unroll
        for (int dd = 32; dd >= 1; dd >>= 1) {
            o |= (uint64_t)__shfl_xor((unsigned long long)o, dd, WAVE);
            a &= (uint64_t)__shfl_xor((unsigned long long)a, dd, WAVE);
        }
        if (lane == 0) {
            s_or[w] = o;
            s_and[w] = a;
        }
        __syncthreads();
        uint64_t oo = 0, aa = ~0ull;
#pragma unroll
        for (int ww = 0; ww < NW; ++ww) {
            oo |= s_or[ww];
            aa &= s_and[ww];
        }
        __syncthreads();
        return oo ^ aa;
    };
    uint64_t k[ITEMS];
    uint32_t sr[ITEMS], dig[ITEMS], pos[ITEMS];
    // one digit pass of (k, sr) through LDS
    auto pass = [&]() {
        uint32_t bc;
        rank_digits<8, ITEMS, NW>(dig, nvalid, pos, s_whist, s_binstart, s_scan, &bc);
#pragma unroll
        for (int i = 0; i < ITEMS; ++i) {
            s_k[pos[i]] = k[i];
            s_sr[pos[i]] = sr[i];
        }
        __syncthreads();
#pragma unroll
        for (int i = 0; i < ITEMS; ++i) {
            k[i] = s_k[posof(i)];
            sr[i] = s_sr[posof(i)];
        }
        __syncthreads();
    };
#pragma unroll
    for (int i = 0; i < ITEMS; ++i) {
        const uint32_t p = posof(i);
        k[i] = p < nvalid ? codes[start + p] : ~0ull;
        sr[i] = p;
    }
    // 1. by code
    uint64_t vary = pack_varying(k, vary_of(k));  // (rank.h)
    for (int shift = 0; shift < code_bits; shift += 8) {
        const uint32_t dmask = (1u << min(8, code_bits - shift)) - 1u;
        if (!((uint32_t)(vary >> shift) & dmask)) continue;
#pragma unroll
        for (int i = 0; i < ITEMS; ++i) dig[i] = (uint32_t)(k[i] >> shift) & dmask;
        pass();
    }
    // 2. run starts (items are in code order now)
#pragma unroll
    for (int i = 0; i < ITEMS; ++i) s_k[posof(i)] = k[i];
    __syncthreads();
    bool repeats = false;
    uint32_t t[ITEMS];
#pragma unroll
    for (int i = 0; i < ITEMS; ++i) {
        const uint32_t p = posof(i);
        const bool head = p == 0 || p >= nvalid || s_k[p - 1] != k[i];
        repeats = repeats || !head;
        t[i] = head ? p : 0u;
    }
    repeats = __syncthreads_or(repeats);
    if (repeats) {
        tile_running_max<ITEMS, NW>(t, s_k32, s_scan);
#pragma unroll
        for (int i = 0; i < ITEMS; ++i) sr[i] |= t[i] << 16;
        // 3. by (run start, refinement key), stable in slot
#pragma unroll
        for (int i = 0; i < ITEMS; ++i) {
            k[i] = posof(i) < nvalid ? k0[start + (sr[i] & 0xFFFFu)] : ~0ull;
            // whether the key continues, kept in bit 31 while the keys are packed
            sr[i] |= posof(i) < nvalid && key_continues<CODER>(k[i]) ? 1u << 31 : 0u;
        }
        vary = pack_varying(k, vary_of(k));
        for (int shift = 0; shift < 64; shift += 8) {
            if (!((uint32_t)(vary >> shift) & 0xFFu)) continue;
#pragma unroll
            for (int i = 0; i < ITEMS; ++i) dig[i] = (uint32_t)(k[i] >> shift) & 0xFFu;
            pass();
        }
        for (int shift = 16; shift < 32; shift += 8) {  // run starts are < 2^15
#pragma unroll
            for (int i = 0; i < ITEMS; ++i) dig[i] = (sr[i] >> shift) & (shift == 24 ? 0x7Fu : 0xFFu);
            pass();
        }
        // 4. groups: same run, same key, and the key continues
#pragma unroll
        for (int i = 0; i < ITEMS; ++i) {
            s_k[posof(i)] = k[i];
            s_sr[posof(i)] = sr[i];
        }
        __syncthreads();
        bool tied = false;
#pragma unroll
        for (int i = 0; i < ITEMS; ++i) {
            const uint32_t p = posof(i);
            const bool same = p > 0 && p < nvalid && ((s_sr[p - 1] ^ sr[i]) & 0x7FFF0000u) == 0 &&
                              s_k[p - 1] == k[i] && (sr[i] >> 31);
            tied = tied || same;
            t[i] = same ? 0u : p;
        }
        tied = __syncthreads_or(tied);
        if (tied && threadIdx.x == 0) scan_list[atomicAdd(scan_count, 1u)] = RunItem{start, nvalid, 0u, LCP_NONE};
        tile_running_max<ITEMS, NW>(t, s_k32, s_scan);
    } else {
#pragma unroll
        for (int i = 0; i < ITEMS; ++i) t[i] = posof(i);
    }
    // indices gathered by slot into LDS before any is overwritten
#pragma unroll
    for (int i = 0; i < ITEMS; ++i)
        if (posof(i) < nvalid) s_k32[posof(i)] = perm[start + (sr[i] & 0xFFFFu)];
    __syncthreads();
#pragma unroll
    for (int i = 0; i < ITEMS; ++i) {
        const uint32_t p = posof(i);
        if (p < nvalid) {
            perm[start + p] = s_k32[p];
            codes[start + p] = (uint64_t)start + t[i];
        }
    }
    __syncthreads();  // LDS is reused by the next bucket
    }
}

// ------------------------------------------------------------------ per-bucket sort on packed (code, key)
// The same result as k_bucket_refine for a bucket whose code bits and first
// refinement key bits that vary over the bucket number at most 64 together:
// both are packed to their varying bits (code above key) in one word, and
// one LSD sequence over that word orders the bucket by code, then by key,
// ties in slot (input) order -- k_bucket_refine's order, without its passes
// by run start.  Equal words are exactly equal (code, key) pairs, so the
// groups (equal pair whose key continues) and the tie keys written in place
// of the codes are the same too.  A bucket whose bits do not fit goes to
// `fallback` for k_bucket_refine.
template <int CODER, int ITEMS, int NW>
__global__ __launch_bounds__(NW * WAVE) void k_bucket_pack(uint64_t* __restrict__ codes,
                                                       uint32_t* __restrict__ perm,
                                                       const uint64_t* __restrict__ k0,
                                                       const RunItem* __restrict__ list,
                                                       const uint32_t* __restrict__ list_count,
                                                       RunItem* __restrict__ fallback,
                                                       uint32_t* __restrict__ fallback_count,
                                                       RunItem* __restrict__ scan_list,
                                                       uint32_t* __restrict__ scan_count) {
    constexpr uint32_t TILE = NW * WAVE * ITEMS;
    static_assert(TILE <= 32768, "slots fit 16 bits");
    __shared__ uint64_t s_k[TILE];
    __shared__ uint32_t s_sr[TILE];
    __shared__ uint32_t s_whist[NW * 256];
    __shared__ uint32_t s_binstart[256];
    __shared__ uint32_t s_scan[NW];
    __shared__ uint64_t s_or[NW], s_and[NW], s_or2[NW], s_and2[NW];
    uint32_t* s_k32 = reinterpret_cast<uint32_t*>(s_k);  // scratch while keys sit in registers
    const uint32_t nlist = *list_count;
    const uint32_t w = threadIdx.x / WAVE, lane = lane_id();
    for (uint32_t it = blockIdx.x; it < nlist; it += gridDim.x) {
        const RunItem d = list[it];
        if (d.len < 2 || d.len > TILE) continue;  // never listed so; uniform per workgroup
        const uint32_t nvalid = d.len, start = d.start;
        auto posof = [&](int i) { return w * WAVE * ITEMS + i * WAVE + lane; };
        // per item: key, and slot | key continues << 31
        uint64_t k[ITEMS], q[ITEMS];
        uint32_t sr[ITEMS], dig[ITEMS], pos[ITEMS], t[ITEMS];
#pragma unroll
        for (int i = 0; i < ITEMS; ++i) {
            const uint32_t p = posof(i);
            k[i] = p < nvalid ? codes[start + p] : ~0ull;
            q[i] = p < nvalid ? k0[start + p] : 0ull;
            sr[i] = p | (p < nvalid && key_continues<CODER>(q[i]) ? 1u << 31 : 0u);
        }
        // bits that vary over the bucket, of the codes and of the keys
        uint64_t o = 0, a = ~0ull, o2 = 0, a2 = ~0ull;
#pragma unroll
        for (int i = 0; i < ITEMS; ++i)
            if (posof(i) < nvalid) {
                o |= k[i];
                a &= k[i];
                o2 |= q[i];
                a2 &= q[i];
            }
#pragma unroll
        for (int dd = 32; dd >= 1; dd >>= 1) {
            o |= (uint64_t)__shfl_xor((unsigned long long)o, dd, WAVE);
            a &= (uint64_t)__shfl_xor((unsigned long long)a, dd, WAVE);
            o2 |= (uint64_t)__shfl_xor((unsigned long long)o2, dd, WAVE);
            a2 &= (uint64_t)__shfl_xor((unsigned long long)a2, dd, WAVE);
        }
        if (lane == 0) {
            s_or[w] = o;
            s_and[w] = a;
            s_or2[w] = o2;
            s_and2[w] = a2;
        }
        __syncthreads();
        uint64_t vc = 0, vq = 0;
        {
            uint64_t oo = 0, aa = ~0ull, oo2 = 0, aa2 = ~0ull;
#pragma unroll
            for (int ww = 0; ww < NW; ++ww) {
                oo |= s_or[ww];
                aa &= s_and[ww];
                oo2 |= s_or2[ww];
                aa2 &= s_and2[ww];
            }
            vc = oo ^ aa;
            vq = oo2 ^ aa2;
        }
        __syncthreads();
        const int cb = __popcll(vc), kb = __popcll(vq);
        if (cb + kb > 64) {
            if (threadIdx.x == 0) fallback[atomicAdd(fallback_count, 1u)] = d;
            continue;
        }
        pack_bits(q, vq);  // (rank.h)
        pack_bits(k, vc);
#pragma unroll
        for (int i = 0; i < ITEMS; ++i) k[i] = (kb >= 64 ? 0ull : k[i] << kb) | q[i];
        // LSD passes over the packed word (every packed bit varies)
        for (int shift = 0; shift < cb + kb; shift += 8) {
#pragma unroll
            for (int i = 0; i < ITEMS; ++i) dig[i] = (uint32_t)(k[i] >> shift) & 0xFFu;
            uint32_t bc;
            rank_digits<8, ITEMS, NW>(dig, nvalid, pos, s_whist, s_binstart, s_scan, &bc);
#pragma unroll
            for (int i = 0; i < ITEMS; ++i) {
                s_k[pos[i]] = k[i];
                s_sr[pos[i]] = sr[i];
            }
            __syncthreads();
#pragma unroll
            for (int i = 0; i < ITEMS; ++i) {
                k[i] = s_k[posof(i)];
                sr[i] = s_sr[posof(i)];
            }
            __syncthreads();
        }
        // groups: equal words whose key continues; tie key = first position
#pragma unroll
        for (int i = 0; i < ITEMS; ++i) s_k[posof(i)] = k[i];
        __syncthreads();
        bool tied = false;
#pragma unroll
        for (int i = 0; i < ITEMS; ++i) {
            const uint32_t p = posof(i);
            const bool same = p > 0 && p < nvalid && s_k[p - 1] == k[i] && (sr[i] >> 31);
            tied = tied || same;
            t[i] = same ? 0u : p;
        }
        tied = __syncthreads_or(tied);
        if (tied) {
            if (threadIdx.x == 0) scan_list[atomicAdd(scan_count, 1u)] = RunItem{start, nvalid, 0u, LCP_NONE};
            tile_running_max<ITEMS, NW>(t, s_k32, s_scan);
        }
        // indices gathered by slot into LDS before any is overwritten
#pragma unroll
        for (int i = 0; i < ITEMS; ++i)
            if (posof(i) < nvalid) s_k32[posof(i)] = perm[start + (sr[i] & 0xFFFFu)];
        __syncthreads();
#pragma unroll
        for (int i = 0; i < ITEMS; ++i) {
            const uint32_t p = posof(i);
            if (p < nvalid) {
                perm[start + p] = s_k32[p];
                codes[start + p] = (uint64_t)start + t[i];
            }
        }
        __syncthreads();  // LDS is reused by the next bucket
    }
}

hipError_t learned_bucket_refine(int coder, uint64_t* codes, uint32_t* perm, const uint64_t* k0,
                                 RunItem* const lists[4], const uint32_t* counts,
                                 RunItem* const fallback[4], uint32_t* fallback_counts,
                                 RunItem* scan_list, uint32_t* scan_count, int c_begin, int c_end,
                                 hipStream_t s) {
    ProfScope ps(P_TILE_SORT, s);
    // four size classes (bucket lists built by k_bucket_classes); a smaller
    // class needs fewer registers and less LDS, so more workgroups share a
    // CU, and wastes fewer padding slots; persistent workgroups walk a list
    uint32_t cus = 256;
    {
        int dev = 0, v = 0;
        if (hipGetDevice(&dev) == hipSuccess &&
            hipDeviceGetAttribute(&v, hipDeviceAttributeMultiprocessorCount, dev) == hipSuccess && v > 0)
            cus = (uint32_t)v;
    }
    // per class: buckets whose (code, key) bits fit one word on the packed
    // path, the others on the general one
#define HUSKY_RF(C, I, NW, L, PER_CU, BITS)                                                           \
    if (L >= c_begin && L < c_end) {                                                                  \
        hipLaunchKernelGGL((k_bucket_pack<C, I, NW>), dim3(cus * PER_CU), dim3(NW * WAVE), 0, s,      \
                           codes, perm, k0, (const RunItem*)lists[L], counts + L, fallback[L],        \
                           fallback_counts + L, scan_list, scan_count);                              \
        hipLaunchKernelGGL((k_bucket_refine<C, I, NW>), dim3(cus * PER_CU), dim3(NW * WAVE), 0, s,    \
                           codes, perm, k0, (const RunItem*)fallback[L], fallback_counts + L, BITS,  \
                           scan_list, scan_count);                                                   \
    }
    // element kind 0 (bytes) or 1 (UTF-16 units); the ASCII code's top bit is
    // always clear, the other coders use all 64
    if (coder == CODER_ASCII7) {
        HUSKY_RF(0, 12, 4, 0, 4, 63);
        HUSKY_RF(0, 16, 4, 1, 3, 63);
        HUSKY_RF(0, 12, 8, 2, 2, 63);
        HUSKY_RF(0, 16, 8, 3, 1, 63);
    } else if (coder == CODER_BYTES8) {
        HUSKY_RF(0, 12, 4, 0, 4, 64);
        HUSKY_RF(0, 16, 4, 1, 3, 64);
        HUSKY_RF(0, 12, 8, 2, 2, 64);
        HUSKY_RF(0, 16, 8, 3, 1, 64);
    } else {
        HUSKY_RF(1, 12, 4, 0, 4, 64);
        HUSKY_RF(1, 16, 4, 1, 3, 64);
        HUSKY_RF(1, 12, 8, 2, 2, 64);
        HUSKY_RF(1, 16, 8, 3, 1, 64);
    }
#undef HUSKY_RF
    return hipGetLastError();
}

// ------------------------------------------------------------------ host side
size_t learned_model_bytes() {
    size_t off[N_PARTS + 1];
    model_offsets(off);
    return off[N_PARTS];
}
size_t learned_model_offset(int part) {
    if (part < 0 || part >= N_PARTS) return ~(size_t)0;
    size_t off[N_PARTS + 1];
    model_offsets(off);
    return off[part];
}
uint32_t learned_nparam() { return NPARAM; }
uint32_t learned_lut_tiles() { return (LUT_CELLS + 1 + LUT_TILE - 1) / LUT_TILE; }

static uint32_t grid_for(uint64_t n, uint32_t cap = 8192) {
    return (uint32_t)std::max<uint64_t>(1, std::min<uint64_t>((n + 255) / 256, cap));
}

hipError_t learned_sample(uint32_t* sel, uint32_t S, uint32_t n, uint64_t seed, hipStream_t s) {
    hipLaunchKernelGGL(k_sample_idx, dim3(grid_for(S)), dim3(256), 0, s, sel, S, n, seed);
    return hipGetLastError();
}

hipError_t learned_prepare(void* model, const uint64_t* sorted_sample, uint32_t S, uint32_t mode,
                           uint32_t flags, uint8_t* fl, uint2* tsum, float* x, float* y,
                           hipStream_t s) {
    ModelView m = model_view(model);
    hipLaunchKernelGGL(k_learned_header, dim3(1), dim3(1), 0, s, sorted_sample, S, m.hdr, mode, flags);
    const uint32_t use_dense = (flags & HUSKY_LEARNED_NO_DENSE) ? 0u : 1u;
    hipLaunchKernelGGL(k_dense_flags, dim3(grid_for(S)), dim3(256), 0, s, sorted_sample, S,
                       (const LearnedHeader*)m.hdr, use_dense, fl);
    const uint32_t tiles = (S + SCAN_TILE - 1) / SCAN_TILE;
    hipLaunchKernelGGL(k_flag_sums, dim3(tiles), dim3(256), 0, s, (const uint8_t*)fl, S, tsum);
    hipLaunchKernelGGL(k_flag_scan, dim3(1), dim3(256), 0, s, tsum, tiles, m.hdr);
    hipLaunchKernelGGL(k_flag_apply, dim3(tiles), dim3(256), 0, s, (const uint8_t*)fl, sorted_sample, S,
                       (const uint2*)tsum, (const LearnedHeader*)m.hdr, x, y, m.dense, m.dense_cum);
    return hipGetLastError();
}

const uint32_t* learned_dense_keys_ptr(void* model) { return &model_view(model).hdr->dense_keys; }

hipError_t learned_init(void* model, uint64_t seed, bool raw, hipStream_t s) {
    ModelView m = model_view(model);
    hipLaunchKernelGGL(k_mlp_init, dim3((NPARAM + 255) / 256), dim3(256), 0, s, m.params, m.adam_m,
                       m.adam_v, seed, raw ? 1 : 0);
    return hipGetLastError();
}


template <bool MONO>
static hipError_t mlp_grad_launch(const float* params, const float* x, const float* y,
                                  uint32_t first, uint32_t count, uint32_t stride, uint32_t blocks,
                                  float inv_batch, float* partial, float* grad, hipStream_t s) {
    const uint32_t per_block = (count + blocks - 1) / blocks;
    hipLaunchKernelGGL(k_mlp_grad<MONO>, dim3(blocks), dim3(MLP_T), 0, s, params, x, y, first,
                       count, stride, per_block, inv_batch, partial);
    hipLaunchKernelGGL(k_mlp_reduce, dim3((NPARAM + 1 + 255) / 256), dim3(256), 0, s,
                       (const float*)partial, blocks, grad);
    return hipGetLastError();
}

static uint32_t grad_blocks(uint32_t count, uint32_t max_blocks) {
    return std::max(1u, std::min(max_blocks, (count + MLP_T - 1) / MLP_T));
}
size_t learned_partial_bytes(uint32_t max_blocks) { return (size_t)max_blocks * (NPARAM + 1) * 4; }

hipError_t learned_grad(const float* params, const float* x, const float* y, uint32_t count,
                        bool mono, float* partial, uint32_t max_blocks, float* grad, hipStream_t s) {
    const uint32_t blocks = grad_blocks(count, max_blocks);
    const float inv = 1.f / (float)std::max(count, 1u);
    return mono ? mlp_grad_launch<true>(params, x, y, 0, count, 1, blocks, inv, partial, grad, s)
                : mlp_grad_launch<false>(params, x, y, 0, count, 1, blocks, inv, partial, grad, s);
}

hipError_t learned_train(void* model, const float* x, const float* y, uint32_t count,
                         uint32_t epochs, uint32_t batch, float lr, bool mono, float* partial,
                         uint32_t max_blocks, float* grad, float* loss_acc, hipStream_t s) {
    ModelView m = model_view(model);
    const float b1 = 0.9f, b2 = 0.999f, eps = 1e-8f;
    uint32_t step = 0;
    hipError_t e = hipSuccess;
    if (count) {
        const uint32_t nb = std::max(1u, (count + batch - 1) / batch);  // batches per epoch
        for (uint32_t ep = 0; ep < epochs; ++ep) {
            if ((e = zero_u32((uint32_t*)loss_acc, 1, s)) != hipSuccess) return e;
            for (uint32_t b = 0; b < nb; ++b) {
                // batch b takes samples b, b + nb, b + 2 nb, ...: every batch
                // spans the whole key range
                const uint32_t cnt = (count - b + nb - 1) / nb;
                const uint32_t blocks = grad_blocks(cnt, max_blocks);
                const float inv = 1.f / (float)cnt;
                e = mono ? mlp_grad_launch<true>(m.params, x, y, b, cnt, nb, blocks, inv, partial, grad, s)
                         : mlp_grad_launch<false>(m.params, x, y, b, cnt, nb, blocks, inv, partial, grad, s);
                if (e != hipSuccess) return e;
                ++step;
                const float c1 = 1.f - powf(b1, (float)step), c2 = 1.f - powf(b2, (float)step);
                hipLaunchKernelGGL(k_adam, dim3((NPARAM + 255) / 256), dim3(256), 0, s, m.params,
                                   m.adam_m, m.adam_v, (const float*)grad, lr, b1, b2, eps, c1, c2,
                                   loss_acc);
            }
        }
    }
    hipLaunchKernelGGL(k_learned_finish, dim3(1), dim3(1), 0, s, m.hdr, (const float*)loss_acc, step,
                       step ? count : 0u);
    return hipGetLastError();
}

hipError_t learned_eval_lut(const float* p, const void* model, uint32_t mode, uint32_t* lut,
                            uint32_t* tmax, hipStream_t s) {
    ModelView m = model_view(const_cast<void*>(model));
    const LearnedHeader* h = m.hdr;
    const dim3 g(8192), t(256);
    switch (mode) {
        case HUSKY_LEARNED_EQUAL_WIDTH:
            hipLaunchKernelGGL((k_lut_eval<LUT_IDENTITY>), g, t, 0, s, h, m.dense, m.dense_cum, lut);
            break;
        case HUSKY_LEARNED_CONSTANT:
            hipLaunchKernelGGL((k_lut_eval<LUT_ZERO>), g, t, 0, s, h, m.dense, m.dense_cum, lut);
            break;
        case HUSKY_LEARNED_UNCONSTRAINED:
            hipLaunchKernelGGL((k_lut_net<false>), dim3(2048), t, 0, s, p, h, m.dense, m.dense_cum, lut);
            break;
        default:
            hipLaunchKernelGGL((k_lut_net<true>), dim3(2048), t, 0, s, p, h, m.dense, m.dense_cum, lut);
    }
    const uint32_t n = LUT_CELLS + 1, tiles = (n + LUT_TILE - 1) / LUT_TILE;
    hipLaunchKernelGGL(k_lut_tilemax, dim3(tiles), dim3(256), 0, s, (const uint32_t*)lut, n, tmax);
    hipLaunchKernelGGL(k_lut_carry, dim3(1), dim3(256), 0, s, tmax, tiles);
    hipLaunchKernelGGL(k_lut_apply, dim3(tiles), dim3(256), 0, s, lut, n, (const uint32_t*)tmax);
    return hipGetLastError();
}

hipError_t learned_build_lut(void* model, uint32_t mode, uint32_t* tmax, hipStream_t s) {
    ModelView m = model_view(model);
    return learned_eval_lut(m.params, model, mode, m.lut, tmax, s);
}

hipError_t learned_splitters(void* model, const uint64_t* sorted_sample, uint32_t S, hipStream_t s) {
    ModelView m = model_view(model);
    hipLaunchKernelGGL(k_splitters, dim3(8192), dim3(256), 0, s, (const uint32_t*)m.lut, sorted_sample,
                       S, m.hdr, m.splitters);
    hipLaunchKernelGGL(k_subtables, dim3(grid_for((uint64_t)SUB_SLOT * LEARNED_BUCKETS)), dim3(256), 0, s,
                       (const uint32_t*)m.lut, (const LearnedHeader*)m.hdr,
                       (const uint64_t*)m.splitters, m.subtab);
    hipLaunchKernelGGL(k_cellinfo, dim3(8192), dim3(256), 0, s, (const uint32_t*)m.lut,
                       (const LearnedHeader*)m.hdr, (const uint64_t*)m.splitters, m.cellinfo);
    return hipGetLastError();
}

BucketArgs learned_bucket_args(const void* model, uint16_t* bid) {
    ModelView m = model_view((void*)model);
    return BucketArgs{m.hdr, m.cellinfo, m.splitters, m.subtab, bid};
}

hipError_t learned_bucket_pass(int pass, const uint64_t* ks, const uint32_t* vs, const uint16_t* bs,
                               const uint64_t* k0s, uint64_t* kd, uint32_t* vd, uint16_t* bd,
                               uint64_t* k0d, uint32_t n, uint32_t* cnt, uint32_t* gtot,
                               uint32_t* binstart, hipStream_t s) {
    constexpr int ITEMS = 16;
    constexpr uint32_t TILE = BLOCK * ITEMS;
    const uint32_t tiles = (n + TILE - 1) / TILE, groups = (tiles + GROUP_TILES - 1) / GROUP_TILES;
    const int shift = 8 * pass;
    {
        ProfScope ps(P_COUNT_SCAN, s);
        hipLaunchKernelGGL(k_bcount<ITEMS>, dim3(tiles), dim3(BLOCK), 0, s, bs, n, shift, cnt);
        hipLaunchKernelGGL(k_lgroup_scan, dim3(groups), dim3(256), 0, s, cnt, tiles, gtot);
        hipLaunchKernelGGL(k_lseg_scan, dim3(1), dim3(256), 0, s, gtot, groups, binstart);
    }
    // timed (when profiling) by events that the dispatch itself records
    hipEvent_t ev0, ev1;
    ProfScope ps(P_BUCKET, s, &ev0, &ev1);
    if (k0s)
        hipExtLaunchKernelGGL((k_bscatter<ITEMS, true>), dim3(tiles), dim3(BLOCK), 0, s, ev0, ev1, 0u,
                              ks, vs, bs, k0s, kd, vd, bd, k0d, n, shift, (const uint32_t*)cnt,
                              (const uint32_t*)gtot, (const uint32_t*)binstart);
    else
        hipExtLaunchKernelGGL((k_bscatter<ITEMS, false>), dim3(tiles), dim3(BLOCK), 0, s, ev0, ev1, 0u,
                              ks, vs, bs, k0s, kd, vd, bd, k0d, n, shift, (const uint32_t*)cnt,
                              (const uint32_t*)gtot, (const uint32_t*)binstart);
    return hipGetLastError();
}
uint32_t learned_pass_tiles(uint32_t n) { return (n + BLOCK * 16 - 1) / (BLOCK * 16); }

hipError_t learned_bucket_bounds(const uint16_t* bid, uint32_t n, uint64_t* seg, uint32_t* overflow,
                                 RunItem* big_list, uint32_t* big_count, RunItem* scan_list,
                                 uint32_t* scan_count, RunItem* const lists[4],
                                 uint32_t* class_count, hipStream_t s) {
    ProfScope ps(P_BUCKET_BOUNDS, s);
    hipLaunchKernelGGL(k_bucket_bounds, dim3(grid_for((uint64_t)n / 8 + 1)), dim3(256), 0, s, bid, n,
                       (uint32_t)LEARNED_BUCKETS, seg);
    hipLaunchKernelGGL(k_bucket_classes, dim3(256), dim3(256), 0, s, (const uint64_t*)seg,
                       (uint32_t)LEARNED_BUCKETS, overflow, big_list, big_count, scan_list, scan_count,
                       lists[0], lists[1], lists[2], lists[3], class_count);
    return hipGetLastError();
}

}  // namespace husky
