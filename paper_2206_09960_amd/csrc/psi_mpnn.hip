// Learned warm start of Power-ψ: the message-passing network's kernels.
//
// The fixed point of eq. (power_psi), s = Aᵀs + c with A ≥ 0 entrywise
// (Sec. II), satisfies s ≥ c, so a start s0 = c ⊙ exp(t̂) with t̂ ≥ 0 lies on
// the right side of c.  The network predicts t̂ ≈ log(s/c) for every user:
//
//   x0 (8 features of activity and degree) → h0 = ReLU(x0 Win + bin)    (64)
//   3 ×:  p_j = (h_j Wm) / den_j                                        (32)
//         m_i = log(1 + ReLU((λ_i + μ_i) Σ_{j∈F(i)} p_j))   (pull pattern of Aᵀ)
//         h   = ReLU([h | m] Wl + bl)                                   (64)
// Dividing eq. (power_psi) by c_i gives log(s_i/c_i) = log(1 + (λ_i + μ_i)
// Σ_{j∈F(i)} s_j/den_j); the receiver factor and the log let one layer
// express that relation.
//   out = h · w_out + b_out,   t̂ = softplus(out)
//
// Algorithm 2 converges from any start (the map contracts to its unique
// fixed point), so a poor prediction costs iterations, never correctness;
// psi_solve also compares the residuals of s0 and c and keeps the better.
//
// Layout and precision.  Activations h (64 wide) and the messages p, m (32
// wide) are stored as bfloat16 rows, 128 B / 64 B per user.  The dense
// products run on MFMA (v_mfma_f32_16x16x32_bf16, FP32 accumulate) with one
// 16-user tile per wave and the bf16 weights held in registers.  The
// aggregation gathers one 64-byte message per edge of CSR(Aᵀ) and sums in
// FP32.  The backward pass is FP32 (bf16 weights and activations enter as
// their exact FP32 values); its aggregation runs over CSR(A).  Every sum
// has a fixed order (weight gradients are per-workgroup partials added in
// workgroup order), so forward and backward are bitwise repeatable.
#include <algorithm>
#include <cmath>

#include "psi_internal.h"

struct psi_model {
  int device = 0;
  float* params = nullptr;  // [kNParam] FP32, order documented in psi.h
  float* adam_m = nullptr;
  float* adam_v = nullptr;
  float* grad = nullptr;
  void* frag = nullptr;     // bf16 MFMA B-fragments of Wm, Wl (per layer)
  int64_t step = 0;         // Adam steps taken
};

namespace psi {
namespace {

typedef __bf16 bf16x8_t __attribute__((ext_vector_type(8)));
typedef float f32x4_t __attribute__((ext_vector_type(4)));
typedef unsigned u32x4_t __attribute__((ext_vector_type(4)));
typedef unsigned u32x2_t __attribute__((ext_vector_type(2)));

// ---------------------------------------------------------------- network shape
constexpr int kF0 = 8, kH = 64, kMsg = 32, kLayers = 3;
constexpr int kLayerSize = kH * kMsg + (kH + kMsg) * kH + kH;  // Wm, Wl, bl
constexpr int kOffWin = 0;
constexpr int kOffBin = kOffWin + kF0 * kH;
constexpr int kOffLayer0 = kOffBin + kH;
constexpr int off_wm(int l) { return kOffLayer0 + l * kLayerSize; }
constexpr int off_wl(int l) { return off_wm(l) + kH * kMsg; }
constexpr int off_bl(int l) { return off_wl(l) + (kH + kMsg) * kH; }
constexpr int kOffWout = kOffLayer0 + kLayers * kLayerSize;
constexpr int kOffBout = kOffWout + kH;
constexpr int kNParam = kOffBout + 1;
static_assert(kNParam == 25409, "parameter count");

// Fragments per layer: 12 of Wl (3 k-steps × 4 column tiles), 4 of Wm (2 × 2);
// one fragment is 64 lanes × 8 bf16.
constexpr int kFragsPerLayer = 16;
constexpr size_t kFragBytes = size_t(kLayers) * kFragsPerLayer * 64 * 16;

// ---------------------------------------------------------------- work split
constexpr int kNodeRows = 64;     // users per workgroup tile of the dense kernels
constexpr int kMaxNodeGrid = 2048;
constexpr int kMaxBwGrid = 256;

inline unsigned grid_for(int64_t n, int block = kBlock) {
  return static_cast<unsigned>((n + block - 1) / block);
}
inline size_t align_up(size_t x) { return (x + 255) / 256 * 256; }

// ---------------------------------------------------------------- bf16
__device__ inline unsigned short f2bf(float x) {
  unsigned u = __float_as_uint(x);
  if ((u & 0x7fffffffu) > 0x7f800000u) return 0x7fc0;  // NaN stays NaN
  u += 0x7fffu + ((u >> 16) & 1u);                    // round to nearest even
  return static_cast<unsigned short>(u >> 16);
}
__device__ inline float bf2f(unsigned short b) { return __uint_as_float(unsigned(b) << 16); }
__device__ inline float bf_lo(unsigned w) { return __uint_as_float(w << 16); }
__device__ inline float bf_hi(unsigned w) { return __uint_as_float(w & 0xffff0000u); }
__device__ inline unsigned bf_pack(float a, float b) {
  return unsigned(f2bf(a)) | (unsigned(f2bf(b)) << 16);
}

// D = A·B + C for a 16×32 A tile and a 32×16 B tile.  Lane l holds row
// l % 16 of A and column l % 16 of B, each with 8 consecutive k values of
// the k-group l / 16; any fixed assignment of k to (group, element) gives
// the same product as long as A and B use the same one.  D: lane l holds
// column l % 16, rows 4 (l / 16) + 0..3.
__device__ inline f32x4_t mfma(u32x4_t a, u32x4_t b, f32x4_t c) {
  return __builtin_amdgcn_mfma_f32_16x16x32_bf16(__builtin_bit_cast(bf16x8_t, a),
                                                 __builtin_bit_cast(bf16x8_t, b), c, 0, 0, 0);
}

__device__ inline float softplus(float o) { return o > 20.f ? o : log1pf(expf(o)); }
__device__ inline float sigmoid(float o) { return 1.f / (1.f + expf(-o)); }

// ---------------------------------------------------------------- operator view
struct OpView {
  int64_t n;
  const int* row_ptr;     // CSR(Aᵀ): followers of each leader
  const int* fm_row_ptr;  // CSR(A): leaders of each follower
  const double *lam, *mu, *c, *d, *invden;
};

// The 8 input features of user r (zeros past the end, so padded rows add
// nothing to any sum).
__device__ inline void features(const OpView& o, int64_t r, float x[kF0]) {
  if (r >= o.n) {
#pragma unroll
    for (int f = 0; f < kF0; ++f) x[f] = 0.f;
    return;
  }
  const double lam = o.lam[r], mu = o.mu[r], iv = o.invden[r];
  x[0] = logf(float(lam));
  x[1] = logf(float(mu) + 1e-12f);
  x[2] = float(o.c[r]);
  x[3] = float(o.d[r]);
  x[4] = log1pf(float(o.row_ptr[r + 1] - o.row_ptr[r]));
  x[5] = log1pf(float(o.fm_row_ptr[r + 1] - o.fm_row_ptr[r]));
  x[6] = iv > 0.0 ? log1pf(float(1.0 / iv)) : 0.f;
  x[7] = logf(float(lam + mu));
}

// ---------------------------------------------------------------- weights
// B-fragments: lane l of fragment (s, t) holds W[32 s + 8 (l / 16) + i][16 t + l % 16], i < 8.
__global__ void k_mp_frags(const float* params, u32x4_t* frag) {
  const int tid = blockIdx.x * blockDim.x + threadIdx.x;
  if (tid >= kLayers * kFragsPerLayer * 64) return;
  const int lane = tid & 63;
  const int f = (tid >> 6) % kFragsPerLayer;
  const int l = (tid >> 6) / kFragsPerLayer;
  const float* W;
  int ncols, s, t;
  if (f < 12) {
    W = params + off_wl(l);
    ncols = kH;
    s = f / 4;
    t = f % 4;
  } else {
    W = params + off_wm(l);
    ncols = kMsg;
    s = (f - 12) / 2;
    t = (f - 12) % 2;
  }
  const int k0 = 32 * s + 8 * (lane >> 4);
  const int col = 16 * t + (lane & 15);
  u32x4_t v;
#pragma unroll
  for (int p = 0; p < 4; ++p)
    v[p] = bf_pack(W[(k0 + 2 * p) * ncols + col], W[(k0 + 2 * p + 1) * ncols + col]);
  frag[tid] = v;
}

__global__ void k_mp_adam(float* p, float* m, float* v, const float* g, int n, float lr, float b1,
                          float b2, float eps, float c1, float c2) {
  const int k = blockIdx.x * blockDim.x + threadIdx.x;
  if (k >= n) return;
  const float gk = g[k];
  const float mk = b1 * m[k] + (1.f - b1) * gk;
  const float vk = b2 * v[k] + (1.f - b2) * gk * gk;
  m[k] = mk;
  v[k] = vk;
  p[k] -= lr * (mk * c1) / (sqrtf(vk * c2) + eps);
}

// ---------------------------------------------------------------- hub schedule
// Rows with more than kMpHubEdges entries ("hubs") are cut into chunks of
// kMpChunkEdges; the list of hubs and the chunk → hub table depend only on
// the operator and are built once per orientation.
__global__ void k_mp_hub_flags(const int* row_ptr, int64_t n, uint32_t* flags) {
  const int64_t i = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
  if (i > n) return;
  flags[i] = (i < n && row_ptr[i + 1] - row_ptr[i] > kMpHubEdges) ? 1u : 0u;
}

__global__ void k_mp_hub_list(const int* row_ptr, int64_t n, const uint32_t* pos, int* hub_rows,
                              uint32_t* nchunk) {
  const int64_t i = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
  if (i >= n) return;
  const int len = row_ptr[i + 1] - row_ptr[i];
  if (len > kMpHubEdges) {
    hub_rows[pos[i]] = static_cast<int>(i);
    nchunk[pos[i]] = static_cast<uint32_t>((len + kMpChunkEdges - 1) / kMpChunkEdges);
  }
}

__global__ void k_mp_chunk_table(const uint32_t* chunk0, int64_t n_hubs, int* chunk_hub) {
  const int64_t h = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
  if (h >= n_hubs) return;
  for (uint32_t c = chunk0[h]; c < chunk0[h + 1]; ++c) chunk_hub[c] = static_cast<int>(h);
}

// ---------------------------------------------------------------- aggregation
// Forward: out_i = bf16(log1p(max((λ_i + μ_i) Σ_{j∈row i} in_j, 0))), in/out
// bf16 [n × 32].
// Backward: out_i = invden_i · Σ_{j∈row i} in_j, in/out FP32 [n × 32].
// Eight lanes carry one 32-vector (4 values each).  A row of at most
// kMpHubEdges entries belongs to one 8-lane group, which loads 16 column
// indices, then issues the 16 gathers, then adds them in edge order; hub
// chunks are summed by a workgroup (16 consecutive edges per group, the 32
// group sums added in group order) and finished per hub in chunk order.
struct AggArgs {
  const int* row_ptr;
  const int* col;
  int64_t n;
  const int* hub_rows;
  const uint32_t* chunk0;
  const int* chunk_hub;
  float* chunk_part;      // [n_chunks × 32]
  const void* in;
  void* out;
  const double* invden;   // backward: row scale
  const double *lam, *mu; // forward: receiver factor λ + μ
};

template <bool BW>
__device__ inline f32x4_t agg_load(const void* in, int64_t j, int q) {
  if constexpr (BW) {
    return *reinterpret_cast<const f32x4_t*>(static_cast<const float*>(in) + j * kMsg + 4 * q);
  } else {
    const u32x2_t u = *reinterpret_cast<const u32x2_t*>(
        static_cast<const unsigned short*>(in) + j * kMsg + 4 * q);
    return f32x4_t{bf_lo(u[0]), bf_hi(u[0]), bf_lo(u[1]), bf_hi(u[1])};
  }
}

template <bool BW>
__device__ inline void agg_store(const AggArgs& a, int64_t r, int q, f32x4_t v) {
  if constexpr (BW) {
    const float iv = float(a.invden[r]);
    *reinterpret_cast<f32x4_t*>(static_cast<float*>(a.out) + r * kMsg + 4 * q) = v * iv;
  } else {
    const float lm = float(a.lam[r] + a.mu[r]);
#pragma unroll
    for (int k = 0; k < 4; ++k) v[k] = log1pf(fmaxf(lm * v[k], 0.f));
    u32x2_t u;
    u[0] = bf_pack(v[0], v[1]);
    u[1] = bf_pack(v[2], v[3]);
    *reinterpret_cast<u32x2_t*>(static_cast<unsigned short*>(a.out) + r * kMsg + 4 * q) = u;
  }
}

// Sum of edges [b, min(b + 16, e1)) into acc, in edge order; b < e1.  Indices
// past the end repeat the last edge (in bounds, not added), so the 16 loads
// issue back to back.
template <bool BW>
__device__ inline void sum16(const AggArgs& a, int b, int e1, int q, f32x4_t& acc) {
  int j[16];
#pragma unroll
  for (int u = 0; u < 16; ++u) j[u] = a.col[min(b + u, e1 - 1)];
  f32x4_t v[16];
#pragma unroll
  for (int u = 0; u < 16; ++u) v[u] = agg_load<BW>(a.in, j[u], q);
#pragma unroll
  for (int u = 0; u < 16; ++u)
    if (b + u < e1) acc += v[u];
}

template <bool BW>
__global__ __launch_bounds__(kBlock) void k_mp_agg_rows(AggArgs a) {
  const int64_t r = (int64_t(blockIdx.x) * kBlock + threadIdx.x) >> 3;
  const int q = threadIdx.x & 7;
  if (r >= a.n) return;  // whole groups leave; no barriers follow
  const int e0 = a.row_ptr[r], e1 = a.row_ptr[r + 1];
  if (e1 - e0 > kMpHubEdges) return;  // a hub: the chunk kernels sum it
  f32x4_t acc = {0.f, 0.f, 0.f, 0.f};
  for (int b = e0; b < e1; b += 16) sum16<BW>(a, b, e1, q, acc);
  agg_store<BW>(a, r, q, acc);
}

// One workgroup per hub chunk; group gi sums edges e0 + 16 gi .. + 15.
template <bool BW>
__global__ __launch_bounds__(kBlock) void k_mp_agg_hubs(AggArgs a) {
  __shared__ float red[32][kMsg + 1];
  const int gi = threadIdx.x >> 3;
  const int q = threadIdx.x & 7;
  const int ch = blockIdx.x;
  const int h = a.chunk_hub[ch];
  const int r = a.hub_rows[h];
  const int e0 = a.row_ptr[r] + (ch - static_cast<int>(a.chunk0[h])) * kMpChunkEdges;
  const int e1 = min(e0 + kMpChunkEdges, a.row_ptr[r + 1]);
  f32x4_t acc = {0.f, 0.f, 0.f, 0.f};
  const int b = e0 + 16 * gi;
  if (b < e1) sum16<BW>(a, b, e1, q, acc);
#pragma unroll
  for (int u = 0; u < 4; ++u) red[gi][4 * q + u] = acc[u];
  __syncthreads();
  if (threadIdx.x < kMsg) {
    float v = 0.f;
    for (int k = 0; k < 32; ++k) v += red[k][threadIdx.x];
    a.chunk_part[int64_t(ch) * kMsg + threadIdx.x] = v;
  }
}

// One workgroup per hub: 8 slices of its chunks, then the slices in order.
template <bool BW>
__global__ __launch_bounds__(kBlock) void k_mp_agg_hub_finish(AggArgs a) {
  __shared__ float red[8][kMsg];
  const int f = threadIdx.x & 31;
  const int slice = threadIdx.x >> 5;
  const int h = blockIdx.x;
  const int c0 = static_cast<int>(a.chunk0[h]), c1 = static_cast<int>(a.chunk0[h + 1]);
  float v = 0.f;
  for (int c = c0 + slice; c < c1; c += 8) v += a.chunk_part[int64_t(c) * kMsg + f];
  red[slice][f] = v;
  __syncthreads();
  if (threadIdx.x < 8) {
    const int qq = threadIdx.x;
    f32x4_t s = {0.f, 0.f, 0.f, 0.f};
    for (int k = 0; k < 8; ++k)
      s += f32x4_t{red[k][4 * qq], red[k][4 * qq + 1], red[k][4 * qq + 2], red[k][4 * qq + 3]};
    agg_store<BW>(a, a.hub_rows[h], qq, s);
  }
}

// ---------------------------------------------------------------- dense forward
struct MpCtrl {
  double loss_sum;  // Σ over users with c > 0 of (t̂ − t)²
  double n_valid;   // number of users with c > 0
  double loss;      // loss_sum / max(n_valid, 1)
  double pad;
};

struct NodeArgs {
  OpView o;
  const float* params;
  const u32x4_t* frag_wl;  // Wl of this layer (12 fragments × 64 lanes)
  const u32x4_t* frag_wm;  // Wm of the next message (4 fragments × 64 lanes)
  int layer;
  const unsigned short* h_in;  // [n × 64]
  const unsigned short* m_in;  // [n × 32]
  unsigned short* h_out;       // [n × 64]
  unsigned short* msg_out;     // [n × 32]
  float* out_f;                // last layer: out per user (training)
  float* t_hat;                // last layer: t̂ per user (optional)
  double* s0;                  // last layer: c ⊙ exp(t̂) (optional)
  const double* s_target;      // last layer, training: the solver's s
  double* loss_part;           // [grid × 2]
};

// KIND 0: features → h0 → message 0.  KIND 1: [h|m] → h' → next message.
// KIND 2: [h|m] → h3 → out, t̂ (and s0, or the loss terms when TRAIN).
template <int KIND, bool TRAIN>
__global__ __launch_bounds__(kBlock) void k_mp_node(NodeArgs a) {
  __shared__ float xs[4][16][kF0 + 1];
  __shared__ __attribute__((aligned(16))) unsigned short hs[4][16][kH + 8];
  __shared__ __attribute__((aligned(16))) unsigned short ms[4][16][kMsg + 8];
  __shared__ double red[4][2];
  const int lane = threadIdx.x & 63;
  const int w = threadIdx.x >> 6;
  const int colq = lane & 15;  // column within a 16-wide tile
  const int grp = lane >> 4;   // k-group of A/B, row quad of D
  const int64_t n = a.o.n;

  // weights in registers
  u32x4_t wl[12];
  u32x4_t wm[4];
  float bias[4];
  float win[4][kF0];
  float wout[4];
  float bout = 0.f;
  if constexpr (KIND == 0) {
#pragma unroll
    for (int t = 0; t < 4; ++t) {
      bias[t] = a.params[kOffBin + 16 * t + colq];
#pragma unroll
      for (int f = 0; f < kF0; ++f) win[t][f] = a.params[kOffWin + f * kH + 16 * t + colq];
    }
  } else {
#pragma unroll
    for (int f = 0; f < 12; ++f) wl[f] = a.frag_wl[f * 64 + lane];
#pragma unroll
    for (int t = 0; t < 4; ++t) bias[t] = a.params[off_bl(a.layer) + 16 * t + colq];
  }
  if constexpr (KIND < 2) {
#pragma unroll
    for (int f = 0; f < 4; ++f) wm[f] = a.frag_wm[f * 64 + lane];
  } else {
#pragma unroll
    for (int t = 0; t < 4; ++t) wout[t] = a.params[kOffWout + 16 * t + colq];
    bout = a.params[kOffBout];
  }

  double loss = 0.0, cnt = 0.0;
  const int64_t n_tiles = (n + kNodeRows - 1) / kNodeRows;
  for (int64_t tile = blockIdx.x; tile < n_tiles; tile += gridDim.x) {
    const int64_t r0 = tile * kNodeRows + 16 * w;  // first user of this wave's 16
    f32x4_t acc[4];
    if constexpr (KIND == 0) {
      if (lane < 16) {
        float x[kF0];
        features(a.o, r0 + lane, x);
#pragma unroll
        for (int f = 0; f < kF0; ++f) xs[w][lane][f] = x[f];
      }
      __syncthreads();
#pragma unroll
      for (int t = 0; t < 4; ++t)
#pragma unroll
        for (int q = 0; q < 4; ++q) {
          float z = bias[t];
#pragma unroll
          for (int f = 0; f < kF0; ++f) z = fmaf(xs[w][4 * grp + q][f], win[t][f], z);
          acc[t][q] = z;
        }
    } else {
      u32x4_t av[3];
      const int64_t ra = r0 + colq;
      if (ra < n) {
        const u32x4_t* hr = reinterpret_cast<const u32x4_t*>(a.h_in + ra * kH);
        av[0] = hr[grp];
        av[1] = hr[4 + grp];
        av[2] = reinterpret_cast<const u32x4_t*>(a.m_in + ra * kMsg)[grp];
      } else {
        av[0] = av[1] = av[2] = u32x4_t{0u, 0u, 0u, 0u};
      }
#pragma unroll
      for (int t = 0; t < 4; ++t) {
        acc[t] = f32x4_t{bias[t], bias[t], bias[t], bias[t]};
#pragma unroll
        for (int s = 0; s < 3; ++s) acc[t] = mfma(av[s], wl[s * 4 + t], acc[t]);
      }
    }
    // ReLU, bf16, through LDS to row-major order
    unsigned short hb[4][4];
#pragma unroll
    for (int t = 0; t < 4; ++t)
#pragma unroll
      for (int q = 0; q < 4; ++q) {
        const float v = acc[t][q];
        hb[t][q] = f2bf(v > 0.f ? v : (v != v ? v : 0.f));
        hs[w][4 * grp + q][16 * t + colq] = hb[t][q];
      }
    __syncthreads();
    if (KIND < 2 || TRAIN) {  // the last layer's h is kept only for the backward pass
      const int rr = lane >> 2, part = lane & 3;
      const int64_t r = r0 + rr;
      if (r < n) {
        const u32x4_t* src = reinterpret_cast<const u32x4_t*>(&hs[w][rr][16 * part]);
        u32x4_t* dst = reinterpret_cast<u32x4_t*>(a.h_out + r * kH + 16 * part);
        dst[0] = src[0];
        dst[1] = src[1];
      }
    }
    if constexpr (KIND < 2) {
      const u32x4_t a0 = *reinterpret_cast<const u32x4_t*>(&hs[w][colq][8 * grp]);
      const u32x4_t a1 = *reinterpret_cast<const u32x4_t*>(&hs[w][colq][32 + 8 * grp]);
      float iv[4];
#pragma unroll
      for (int q = 0; q < 4; ++q) {
        const int64_t r = r0 + 4 * grp + q;
        iv[q] = r < n ? float(a.o.invden[r]) : 0.f;
      }
#pragma unroll
      for (int t = 0; t < 2; ++t) {
        f32x4_t macc = {0.f, 0.f, 0.f, 0.f};
        macc = mfma(a0, wm[t], macc);
        macc = mfma(a1, wm[2 + t], macc);
#pragma unroll
        for (int q = 0; q < 4; ++q) ms[w][4 * grp + q][16 * t + colq] = f2bf(macc[q] * iv[q]);
      }
      __syncthreads();
      const int rr = lane >> 2, part = lane & 3;
      const int64_t r = r0 + rr;
      if (r < n)
        *reinterpret_cast<u32x4_t*>(a.msg_out + r * kMsg + 8 * part) =
            *reinterpret_cast<const u32x4_t*>(&ms[w][rr][8 * part]);
    } else {
      float p[4];
#pragma unroll
      for (int q = 0; q < 4; ++q) {
        float s = 0.f;
#pragma unroll
        for (int t = 0; t < 4; ++t) s = fmaf(bf2f(hb[t][q]), wout[t], s);
        p[q] = s;
      }
#pragma unroll
      for (int off = 1; off < 16; off <<= 1)
#pragma unroll
        for (int q = 0; q < 4; ++q) p[q] += __shfl_xor(p[q], off, 64);
      if (colq < 4) {
        const float pv = colq == 0 ? p[0] : colq == 1 ? p[1] : colq == 2 ? p[2] : p[3];
        const int64_t r = r0 + 4 * grp + colq;
        if (r < n) {
          const float o = pv + bout;
          const float th = softplus(o);
          if (a.t_hat) a.t_hat[r] = th;
          if (a.s0) a.s0[r] = a.o.c[r] * exp(double(th));
          if constexpr (TRAIN) {
            a.out_f[r] = o;
            const double c = a.o.c[r];
            if (c > 0.0) {
              const double diff = double(th) - log(a.s_target[r] / c);
              loss += diff * diff;
              cnt += 1.0;
            }
          }
        }
      }
    }
    __syncthreads();  // LDS is rewritten by the next tile
  }
  if constexpr (KIND == 2 && TRAIN) {
    for (int off = 32; off > 0; off >>= 1) {
      loss += __shfl_down(loss, off, 64);
      cnt += __shfl_down(cnt, off, 64);
    }
    if (lane == 0) {
      red[w][0] = loss;
      red[w][1] = cnt;
    }
    __syncthreads();
    if (threadIdx.x == 0) {
      a.loss_part[2 * blockIdx.x] = (red[0][0] + red[1][0]) + (red[2][0] + red[3][0]);
      a.loss_part[2 * blockIdx.x + 1] = (red[0][1] + red[1][1]) + (red[2][1] + red[3][1]);
    }
  }
}

__global__ __launch_bounds__(kBlock) void k_mp_loss_reduce(const double* part, int grid,
                                                           MpCtrl* ctrl) {
  __shared__ double rl[kBlock], rc[kBlock];
  double l = 0.0, c = 0.0;
  for (int b = threadIdx.x; b < grid; b += kBlock) {
    l += part[2 * b];
    c += part[2 * b + 1];
  }
  rl[threadIdx.x] = l;
  rc[threadIdx.x] = c;
  __syncthreads();
  for (int s = kBlock / 2; s > 0; s >>= 1) {
    if (threadIdx.x < s) {
      rl[threadIdx.x] += rl[threadIdx.x + s];
      rc[threadIdx.x] += rc[threadIdx.x + s];
    }
    __syncthreads();
  }
  if (threadIdx.x == 0) {
    ctrl->loss_sum = rl[0];
    ctrl->n_valid = rc[0];
    ctrl->loss = rl[0] / fmax(rc[0], 1.0);
  }
}

// ---------------------------------------------------------------- backward
// Per layer l (top first), with G = ∂loss/∂h_{l+1}:
//   G  = d_out w_outᵀ                          (top)
//   G  = dhp + dmsg Wm_{l+1}ᵀ,  ∂Wm_{l+1} += h_{l+1}ᵀ dmsg   (below the top)
//   dz = G ⊙ [h_{l+1} > 0];  ∂Wl_l += [h_l | m_l]ᵀ dz;  ∂bl_l += Σ dz
//   [dhp | dm] = dz Wl_lᵀ,  dm ← dm ⊙ (λ + μ) ⊙ exp(−m_l) ⊙ [m_l > 0]
//   (m = log1p(a) ⇒ dm/da = exp(−m) where a > 0)
// then dmsg = invden ⊙ (Pᵀ dm) by the aggregation over CSR(A).  The input
// kernel finishes with G_0, ∂Wm_0, dz_0 = G_0 ⊙ [h_0 > 0], ∂Win, ∂bin.
struct BwArgs {
  OpView o;
  const float* params;
  int layer;
  const unsigned short* h_in;    // h_l      [n × 64]
  const unsigned short* m_in;    // m_l      [n × 32]
  const unsigned short* h_next;  // h_{l+1}  [n × 64] (the input kernel: h_0)
  const float* dhp_in;           // [n × 64]
  const float* dmsg_in;          // [n × 32]
  const float* out_f;            // top: network output
  const double* s_target;        // top
  const MpCtrl* ctrl;            // top: n_valid
  float* dhp_out;                // [n × 64]
  float* dm_out;                 // [n × 32]
  float* part;                   // [grid × kNParam]
};

__device__ inline void load_bf16_row16(const unsigned short* src, float* dst) {
  const u32x4_t* s = reinterpret_cast<const u32x4_t*>(src);
#pragma unroll
  for (int v = 0; v < 2; ++v) {
    const u32x4_t u = s[v];
#pragma unroll
    for (int p = 0; p < 4; ++p) {
      dst[8 * v + 2 * p] = bf_lo(u[p]);
      dst[8 * v + 2 * p + 1] = bf_hi(u[p]);
    }
  }
}

// MODE 0: top layer.  MODE 1: a layer below the top.  MODE 2: the input layer.
template <int MODE>
__global__ __launch_bounds__(kBlock) void k_mp_bw(BwArgs a) {
  __shared__ __attribute__((aligned(16))) float WlT[kH][kH + kMsg];  // WlT[j][i] = Wl[i][j]
  __shared__ __attribute__((aligned(16))) float WmT[kMsg][kH];       // WmT[k][i] = Wm[i][k]
  __shared__ __attribute__((aligned(16))) float xs[kNodeRows][100];  // [h_l | m_l], then dx
  __shared__ float hn[kNodeRows][kH + 1];
  __shared__ float gz[kNodeRows][kH + 1];
  __shared__ float dms[kNodeRows][kMsg + 1];
  __shared__ float dout_s[kNodeRows];
  __shared__ float xf[kNodeRows][kF0];
  const int t = threadIdx.x;
  const int w = t >> 6;
  const int lane = t & 63;
  const int64_t n = a.o.n;
  const int l = a.layer;
  const int wm_layer = MODE == 2 ? 0 : l + 1;

  // bf16-rounded weights, as the forward pass used them
  if constexpr (MODE != 2) {
    for (int k = t; k < (kH + kMsg) * kH; k += kBlock) {
      const int i = k / kH, j = k % kH;
      WlT[j][i] = bf2f(f2bf(a.params[off_wl(l) + k]));
    }
  }
  if constexpr (MODE != 0) {
    for (int k = t; k < kH * kMsg; k += kBlock) {
      const int i = k / kMsg, kk = k % kMsg;
      WmT[kk][i] = bf2f(f2bf(a.params[off_wm(wm_layer) + k]));
    }
  }
  float inv_valid = 0.f;
  if constexpr (MODE == 0) inv_valid = float(1.0 / fmax(a.ctrl->n_valid, 1.0));

  float pWl[24];   // ∂Wl[24 w + u][lane]          (MODE 0, 1)
  float pWm[8];    // ∂Wm[(t >> 5) + 8 u][t & 31]  (MODE 1, 2)
  float pWin[2];   // ∂Win[2 w + u][lane]          (MODE 2)
  float pb = 0.f;  // ∂bl[lane] / ∂bin[lane] (wave 0)
  float pwout = 0.f, pbout = 0.f;
#pragma unroll
  for (int u = 0; u < 24; ++u) pWl[u] = 0.f;
#pragma unroll
  for (int u = 0; u < 8; ++u) pWm[u] = 0.f;
  pWin[0] = pWin[1] = 0.f;
  __syncthreads();

  const int64_t n_tiles = (n + kNodeRows - 1) / kNodeRows;
  for (int64_t tile = blockIdx.x; tile < n_tiles; tile += gridDim.x) {
    const int64_t base = tile * kNodeRows;
    {  // loads: thread t covers row t / 4, quarter t % 4
      const int rr = t >> 2, qq = t & 3;
      const int64_t r = base + rr;
      const bool ok = r < n;
      float tmp[16];
      if constexpr (MODE != 2) {
        if (ok) load_bf16_row16(a.h_in + r * kH + 16 * qq, tmp);
#pragma unroll
        for (int u = 0; u < 16; ++u) xs[rr][16 * qq + u] = ok ? tmp[u] : 0.f;
        if (ok) {
          const u32x4_t u4 = reinterpret_cast<const u32x4_t*>(a.m_in + r * kMsg)[qq];
#pragma unroll
          for (int p = 0; p < 4; ++p) {
            xs[rr][kH + 8 * qq + 2 * p] = bf_lo(u4[p]);
            xs[rr][kH + 8 * qq + 2 * p + 1] = bf_hi(u4[p]);
          }
        } else {
#pragma unroll
          for (int u = 0; u < 8; ++u) xs[rr][kH + 8 * qq + u] = 0.f;
        }
      }
      if (ok) load_bf16_row16(a.h_next + r * kH + 16 * qq, tmp);
#pragma unroll
      for (int u = 0; u < 16; ++u) hn[rr][16 * qq + u] = ok ? tmp[u] : 0.f;
      if constexpr (MODE != 0) {
#pragma unroll
        for (int v = 0; v < 4; ++v) {
          const f32x4_t g4 = ok ? reinterpret_cast<const f32x4_t*>(a.dhp_in + r * kH + 16 * qq)[v]
                                : f32x4_t{0.f, 0.f, 0.f, 0.f};
#pragma unroll
          for (int p = 0; p < 4; ++p) gz[rr][16 * qq + 4 * v + p] = g4[p];
        }
#pragma unroll
        for (int v = 0; v < 2; ++v) {
          const f32x4_t g4 = ok ? reinterpret_cast<const f32x4_t*>(a.dmsg_in + r * kMsg + 8 * qq)[v]
                                : f32x4_t{0.f, 0.f, 0.f, 0.f};
#pragma unroll
          for (int p = 0; p < 4; ++p) dms[rr][8 * qq + 4 * v + p] = g4[p];
        }
      }
      if constexpr (MODE == 0) {
        if (t < kNodeRows) {
          const int64_t r2 = base + t;
          float dout = 0.f;
          if (r2 < n) {
            const double c = a.o.c[r2];
            if (c > 0.0) {
              const float o = a.out_f[r2];
              const double diff = double(softplus(o)) - log(a.s_target[r2] / c);
              dout = float(2.0 * diff) * inv_valid * sigmoid(o);
            }
          }
          dout_s[t] = dout;
        }
      }
      if constexpr (MODE == 2) {
        if (t < kNodeRows) {
          float x[kF0];
          features(a.o, base + t, x);
#pragma unroll
          for (int f = 0; f < kF0; ++f) xf[t][f] = x[f];
        }
      }
    }
    __syncthreads();
    const int r = lane;  // row owned in the per-row phases
    if constexpr (MODE == 0) {
      // ∂w_out, ∂b_out, and dz = d_out w_outᵀ ⊙ [h3 > 0] (wave w owns columns 16w..16w+15)
      if (w == 0) {
        for (int rr = 0; rr < kNodeRows; ++rr) pwout = fmaf(hn[rr][lane], dout_s[rr], pwout);
        if (lane == 0)
          for (int rr = 0; rr < kNodeRows; ++rr) pbout += dout_s[rr];
      }
      const float d = dout_s[r];
#pragma unroll
      for (int u = 0; u < 16; ++u) {
        const int i = 16 * w + u;
        const float wo = a.params[kOffWout + i];
        gz[r][i] = hn[r][i] > 0.f ? d * wo : 0.f;
      }
    } else {
      // ∂Wm += h_nextᵀ dmsg
      {
        const int kk = t & 31, i0 = t >> 5;
        for (int rr = 0; rr < kNodeRows; ++rr) {
          const float dk = dms[rr][kk];
#pragma unroll
          for (int u = 0; u < 8; ++u) pWm[u] = fmaf(hn[rr][i0 + 8 * u], dk, pWm[u]);
        }
      }
      // G = dhp + dmsg Wmᵀ, then dz = G ⊙ [h_next > 0]
      float g[16];
#pragma unroll
      for (int u = 0; u < 16; ++u) g[u] = gz[r][16 * w + u];
      for (int kk = 0; kk < kMsg; ++kk) {
        const float dk = dms[r][kk];
        const f32x4_t* wr = reinterpret_cast<const f32x4_t*>(&WmT[kk][16 * w]);
#pragma unroll
        for (int v = 0; v < 4; ++v) {
          const f32x4_t wv = wr[v];
#pragma unroll
          for (int p = 0; p < 4; ++p) g[4 * v + p] = fmaf(dk, wv[p], g[4 * v + p]);
        }
      }
#pragma unroll
      for (int u = 0; u < 16; ++u) gz[r][16 * w + u] = hn[r][16 * w + u] > 0.f ? g[u] : 0.f;
    }
    __syncthreads();
    if constexpr (MODE != 2) {
      // ∂Wl += xᵀ dz (thread: column lane, rows 24w..24w+23), ∂bl (wave 0)
      for (int rr = 0; rr < kNodeRows; ++rr) {
        const float dz = gz[rr][lane];
        const f32x4_t* xr = reinterpret_cast<const f32x4_t*>(&xs[rr][24 * w]);
#pragma unroll
        for (int v = 0; v < 6; ++v) {
          const f32x4_t xv = xr[v];
#pragma unroll
          for (int p = 0; p < 4; ++p) pWl[4 * v + p] = fmaf(xv[p], dz, pWl[4 * v + p]);
        }
        if (w == 0) pb += dz;
      }
      __syncthreads();
      // dx = dz Wlᵀ (thread: row lane, outputs 24w..24w+23), into xs
      float dx[24];
#pragma unroll
      for (int u = 0; u < 24; ++u) dx[u] = 0.f;
      for (int j = 0; j < kH; ++j) {
        const float dz = gz[r][j];
        const f32x4_t* wr = reinterpret_cast<const f32x4_t*>(&WlT[j][24 * w]);
#pragma unroll
        for (int v = 0; v < 6; ++v) {
          const f32x4_t wv = wr[v];
#pragma unroll
          for (int p = 0; p < 4; ++p) dx[4 * v + p] = fmaf(dz, wv[p], dx[4 * v + p]);
        }
      }
      // through m = log1p(ReLU((λ + μ) a)): only this thread reads or writes xs[r][24w..24w+23]
      float lm = 0.f;
      if (base + r < n) lm = float(a.o.lam[base + r] + a.o.mu[base + r]);
#pragma unroll
      for (int u = 0; u < 24; ++u) {
        const int i = 24 * w + u;
        if (i >= kH) {
          const float mv = xs[r][i];
          dx[u] = mv > 0.f ? dx[u] * lm * expf(-mv) : 0.f;
        }
        xs[r][i] = dx[u];
      }
      __syncthreads();
      {
        const int rr = t >> 2, qq = t & 3;
        const int64_t rg = base + rr;
        if (rg < n) {
          f32x4_t* dh = reinterpret_cast<f32x4_t*>(a.dhp_out + rg * kH + 16 * qq);
          const f32x4_t* sx = reinterpret_cast<const f32x4_t*>(&xs[rr][16 * qq]);
#pragma unroll
          for (int v = 0; v < 4; ++v) dh[v] = sx[v];
          f32x4_t* dm = reinterpret_cast<f32x4_t*>(a.dm_out + rg * kMsg + 8 * qq);
          const f32x4_t* sm = reinterpret_cast<const f32x4_t*>(&xs[rr][kH + 8 * qq]);
          dm[0] = sm[0];
          dm[1] = sm[1];
        }
      }
    } else {
      // ∂Win += x0ᵀ dz0 (thread: column lane, features 2w, 2w+1), ∂bin (wave 0)
      for (int rr = 0; rr < kNodeRows; ++rr) {
        const float dz = gz[rr][lane];
        pWin[0] = fmaf(xf[rr][2 * w], dz, pWin[0]);
        pWin[1] = fmaf(xf[rr][2 * w + 1], dz, pWin[1]);
        if (w == 0) pb += dz;
      }
    }
    __syncthreads();
  }

  // this workgroup's partial gradient
  float* P = a.part + int64_t(blockIdx.x) * kNParam;
  if constexpr (MODE != 2) {
#pragma unroll
    for (int u = 0; u < 24; ++u) P[off_wl(l) + (24 * w + u) * kH + lane] = pWl[u];
    if (w == 0) P[off_bl(l) + lane] = pb;
  } else {
    P[kOffWin + (2 * w) * kH + lane] = pWin[0];
    P[kOffWin + (2 * w + 1) * kH + lane] = pWin[1];
    if (w == 0) P[kOffBin + lane] = pb;
  }
  if constexpr (MODE != 0) {
    const int kk = t & 31, i0 = t >> 5;
#pragma unroll
    for (int u = 0; u < 8; ++u) P[off_wm(wm_layer) + (i0 + 8 * u) * kMsg + kk] = pWm[u];
  } else {
    if (w == 0) P[kOffWout + lane] = pwout;
    if (t == 0) P[kOffBout] = pbout;
  }
}

__global__ void k_mp_grad_reduce(const float* part, int grid, float* grad) {
  const int k = blockIdx.x * blockDim.x + threadIdx.x;
  if (k >= kNParam) return;
  float s = 0.f;
  for (int b = 0; b < grid; ++b) s += part[int64_t(b) * kNParam + k];
  grad[k] = s;
}

// ---------------------------------------------------------------- workspace
struct MpWs {
  uint32_t* flags;      // [n + 1] hub flags (schedule build)
  uint32_t* scan_tmp;
  uint32_t* scan_total;
  float* chunk_part;    // [max_chunks × 32]
  unsigned short* h[4];
  unsigned short* m[3];
  unsigned short* msg;
  float* out_f;
  float* dhp[2];
  float* dm;
  float* dmsg;
  float* part;
  double* loss_part;
  MpCtrl* ctrl;
  int node_grid, bw_grid;
};

int node_grid_for(int64_t n) {
  return int(std::min<int64_t>((n + kNodeRows - 1) / kNodeRows, kMaxNodeGrid));
}
int bw_grid_for(int64_t n) {
  return int(std::min<int64_t>((n + kNodeRows - 1) / kNodeRows, kMaxBwGrid));
}

size_t mp_layout(const psi_operator* op, bool training, MpWs* w, char* base) {
  const int64_t n = op->n;
  MpWs t{};
  size_t off = 0;
  auto take = [&](size_t bytes) -> char* {
    char* p = base ? base + off : nullptr;
    off += align_up(std::max<size_t>(bytes, 1));
    return p;
  };
  t.flags = (uint32_t*)take(4 * size_t(n + 1));
  const int64_t scan_n = std::max<int64_t>(n + 1, op->mp_max_hubs + 1);
  t.scan_tmp = (uint32_t*)take(4 * size_t(scan_tile_count(scan_n) + 8));
  t.scan_total = (uint32_t*)take(16);
  t.chunk_part = (float*)take(4 * size_t(kMsg) * size_t(op->mp_max_chunks));
  const int n_h = training ? 4 : 2;
  for (int k = 0; k < n_h; ++k) t.h[k] = (unsigned short*)take(2 * size_t(n) * kH);
  const int n_m = training ? 3 : 1;
  for (int k = 0; k < n_m; ++k) t.m[k] = (unsigned short*)take(2 * size_t(n) * kMsg);
  t.msg = (unsigned short*)take(2 * size_t(n) * kMsg);
  t.node_grid = node_grid_for(n);
  t.bw_grid = bw_grid_for(n);
  t.loss_part = (double*)take(16 * size_t(t.node_grid));
  t.ctrl = (MpCtrl*)take(sizeof(MpCtrl));
  if (training) {
    t.out_f = (float*)take(4 * size_t(n));
    t.dhp[0] = (float*)take(4 * size_t(n) * kH);
    t.dhp[1] = (float*)take(4 * size_t(n) * kH);
    t.dm = (float*)take(4 * size_t(n) * kMsg);
    t.dmsg = (float*)take(4 * size_t(n) * kMsg);
    t.part = (float*)take(4 * size_t(t.bw_grid) * kNParam);
  }
  if (w) *w = t;
  return off;
}

// The hub schedule of orientation o (0: CSR(Aᵀ), 1: CSR(A)), built on first
// use and kept in the operator.  Blocks twice to learn the hub and chunk counts.
psi_status ensure_hubs(psi_operator* op, int o, MpWs& w, hipStream_t st) {
  MpHubs& hb = op->mp_hubs[o];
  if (hb.n_hubs >= 0) return PSI_OK;
  const int* row_ptr = o == 0 ? op->row_ptr : op->fm_row_ptr;
  const int64_t n = op->n;
  hipLaunchKernelGGL(k_mp_hub_flags, dim3(grid_for(n + 1)), dim3(kBlock), 0, st, row_ptr, n,
                     w.flags);
  psi_status r = scan_exclusive_u32(w.flags, w.flags, n + 1, w.scan_tmp, w.scan_total, st);
  if (r != PSI_OK) return r;
  uint32_t n_hubs = 0;
  PSI_HIP_CHECK(hipMemcpyAsync(&n_hubs, w.flags + n, 4, hipMemcpyDeviceToHost, st));
  PSI_HIP_CHECK(hipStreamSynchronize(st));
  PSI_REQUIRE(int64_t(n_hubs) <= op->mp_max_hubs, "internal: hub count exceeds its bound");
  uint32_t n_chunks = 0;
  if (n_hubs > 0) {
    hipLaunchKernelGGL(k_mp_hub_list, dim3(grid_for(n)), dim3(kBlock), 0, st, row_ptr, n,
                       w.flags, hb.hub_rows, hb.chunk0);
    PSI_HIP_CHECK(hipMemsetAsync(hb.chunk0 + n_hubs, 0, 4, st));
    r = scan_exclusive_u32(hb.chunk0, hb.chunk0, int64_t(n_hubs) + 1, w.scan_tmp, w.scan_total,
                           st);
    if (r != PSI_OK) return r;
    PSI_HIP_CHECK(hipMemcpyAsync(&n_chunks, hb.chunk0 + n_hubs, 4, hipMemcpyDeviceToHost, st));
    PSI_HIP_CHECK(hipStreamSynchronize(st));
    PSI_REQUIRE(int64_t(n_chunks) <= op->mp_max_chunks, "internal: chunk count exceeds its bound");
    hipLaunchKernelGGL(k_mp_chunk_table, dim3(grid_for(n_hubs)), dim3(kBlock), 0, st, hb.chunk0,
                       int64_t(n_hubs), hb.chunk_hub);
    PSI_HIP_CHECK(hipGetLastError());
  }
  hb.n_hubs = n_hubs;
  hb.n_chunks = n_chunks;
  return PSI_OK;
}

template <bool BW>
psi_status aggregate(const psi_operator* op, int o, MpWs& w, const void* in, void* out,
                     hipStream_t st) {
  const MpHubs& hb = op->mp_hubs[o];
  AggArgs a{o == 0 ? op->row_ptr : op->fm_row_ptr, o == 0 ? op->col : op->fm_col, op->n,
            hb.hub_rows, hb.chunk0, hb.chunk_hub, w.chunk_part, in, out, op->invden, op->lam,
            op->mu};
  hipLaunchKernelGGL(k_mp_agg_rows<BW>, dim3(grid_for(op->n * 8)), dim3(kBlock), 0, st, a);
  if (hb.n_hubs > 0) {
    hipLaunchKernelGGL(k_mp_agg_hubs<BW>, dim3(unsigned(hb.n_chunks)), dim3(kBlock), 0, st, a);
    hipLaunchKernelGGL(k_mp_agg_hub_finish<BW>, dim3(unsigned(hb.n_hubs)), dim3(kBlock), 0, st, a);
  }
  PSI_HIP_CHECK(hipGetLastError());
  return PSI_OK;
}

OpView op_view(const psi_operator* op) {
  return OpView{op->n, op->row_ptr, op->fm_row_ptr, op->lam, op->mu, op->c, op->d, op->invden};
}

const u32x4_t* frag_wl(const psi_model* md, int l) {
  return static_cast<const u32x4_t*>(md->frag) + size_t(l) * kFragsPerLayer * 64;
}
const u32x4_t* frag_wm(const psi_model* md, int l) { return frag_wl(md, l) + 12 * 64; }

// The forward pass; TRAIN keeps every layer's activations and the loss terms.
template <bool TRAIN>
psi_status forward(psi_model* md, psi_operator* op, MpWs& w, float* t_hat, double* s0,
                   const double* s_target, hipStream_t st) {
  psi_status r = ensure_hubs(op, 0, w, st);
  if (r != PSI_OK) return r;
  NodeArgs a{};
  a.o = op_view(op);
  a.params = md->params;
  const dim3 grid(w.node_grid), block(kBlock);
  auto h_at = [&](int k) { return TRAIN ? w.h[k] : w.h[k & 1]; };
  auto m_at = [&](int k) { return TRAIN ? w.m[k] : w.m[0]; };
  // layer 0 input: features → h0, message 0
  a.h_out = h_at(0);
  a.msg_out = w.msg;
  a.frag_wm = frag_wm(md, 0);
  hipLaunchKernelGGL((k_mp_node<0, TRAIN>), grid, block, 0, st, a);
  for (int l = 0; l < kLayers; ++l) {
    r = aggregate<false>(op, 0, w, w.msg, m_at(l), st);
    if (r != PSI_OK) return r;
    a.layer = l;
    a.h_in = h_at(l);
    a.m_in = m_at(l);
    a.h_out = h_at(l + 1);
    a.frag_wl = frag_wl(md, l);
    if (l + 1 < kLayers) {
      a.frag_wm = frag_wm(md, l + 1);
      hipLaunchKernelGGL((k_mp_node<1, TRAIN>), grid, block, 0, st, a);
    } else {
      a.t_hat = t_hat;
      a.s0 = s0;
      a.out_f = w.out_f;
      a.s_target = s_target;
      a.loss_part = w.loss_part;
      hipLaunchKernelGGL((k_mp_node<2, TRAIN>), grid, block, 0, st, a);
    }
  }
  if (TRAIN)
    hipLaunchKernelGGL(k_mp_loss_reduce, dim3(1), dim3(kBlock), 0, st, w.loss_part, w.node_grid,
                       w.ctrl);
  PSI_HIP_CHECK(hipGetLastError());
  return PSI_OK;
}

psi_status backward(psi_model* md, psi_operator* op, MpWs& w, const double* s_target,
                    hipStream_t st) {
  psi_status r = ensure_hubs(op, 1, w, st);
  if (r != PSI_OK) return r;
  BwArgs b{};
  b.o = op_view(op);
  b.params = md->params;
  b.s_target = s_target;
  b.out_f = w.out_f;
  b.ctrl = w.ctrl;
  b.part = w.part;
  b.dm_out = w.dm;
  const dim3 grid(w.bw_grid), block(kBlock);
  for (int l = kLayers - 1; l >= 0; --l) {
    b.layer = l;
    b.h_in = w.h[l];
    b.m_in = w.m[l];
    b.h_next = w.h[l + 1];
    b.dhp_in = w.dhp[(l + 1) & 1];  // written by the layer above (unused at the top)
    b.dmsg_in = w.dmsg;
    b.dhp_out = w.dhp[l & 1];
    if (l == kLayers - 1) hipLaunchKernelGGL(k_mp_bw<0>, grid, block, 0, st, b);
    else hipLaunchKernelGGL(k_mp_bw<1>, grid, block, 0, st, b);
    r = aggregate<true>(op, 1, w, w.dm, w.dmsg, st);
    if (r != PSI_OK) return r;
  }
  b.layer = 0;
  b.h_next = w.h[0];
  b.dhp_in = w.dhp[0];
  b.dmsg_in = w.dmsg;
  hipLaunchKernelGGL(k_mp_bw<2>, grid, block, 0, st, b);
  hipLaunchKernelGGL(k_mp_grad_reduce, dim3(grid_for(kNParam)), dim3(kBlock), 0, st, w.part,
                     w.bw_grid, md->grad);
  PSI_HIP_CHECK(hipGetLastError());
  return PSI_OK;
}

psi_status check_pair(const psi_model* md, const psi_operator* op) {
  PSI_REQUIRE(md && op, "model and op must not be NULL");
  int dev = -1;
  PSI_HIP_CHECK(hipGetDevice(&dev));
  PSI_REQUIRE(dev == op->device && dev == md->device,
              "model, operator and the current device must agree");
  return PSI_OK;
}

psi_status refresh_frags(psi_model* md, hipStream_t st) {
  hipLaunchKernelGGL(k_mp_frags, dim3(grid_for(kLayers * kFragsPerLayer * 64)), dim3(kBlock), 0,
                     st, md->params, static_cast<u32x4_t*>(md->frag));
  PSI_HIP_CHECK(hipGetLastError());
  return PSI_OK;
}

}  // namespace

// ---------------------------------------------------------------- entry points (psi.h)
int64_t mpnn_param_count() { return kNParam; }

size_t model_state_size() { return 4 * align_up(4 * size_t(kNParam)) + kFragBytes; }

psi_status model_create(const float* params, int64_t n_params, uint32_t flags, void* state,
                        size_t state_bytes, hipStream_t st, psi_model** out) {
  PSI_REQUIRE(out, "model must not be NULL");
  *out = nullptr;
  PSI_REQUIRE(params && state, "params and state must not be NULL");
  PSI_REQUIRE(n_params == kNParam, "params must hold psi_mpnn_param_count() values");
  if (state_bytes < model_state_size()) {
    set_error("model state smaller than psi_model_state_size reported");
    return PSI_ENOSPACE;
  }
  int dev = -1;
  PSI_HIP_CHECK(hipGetDevice(&dev));
  const size_t pb = align_up(4 * size_t(kNParam));
  char* b = static_cast<char*>(state);
  const hipMemcpyKind kind = (flags & PSI_INPUT_HOST) ? hipMemcpyHostToDevice
                                                      : hipMemcpyDeviceToDevice;
  PSI_HIP_CHECK(hipMemcpyAsync(b, params, 4 * size_t(kNParam), kind, st));
  PSI_HIP_CHECK(hipMemsetAsync(b + pb, 0, 3 * pb, st));
  hipLaunchKernelGGL(k_mp_frags, dim3(grid_for(kLayers * kFragsPerLayer * 64)), dim3(kBlock), 0,
                     st, reinterpret_cast<const float*>(b), reinterpret_cast<u32x4_t*>(b + 4 * pb));
  PSI_HIP_CHECK(hipGetLastError());
  PSI_HIP_CHECK(hipStreamSynchronize(st));
  psi_model* md = new psi_model();
  md->device = dev;
  md->params = reinterpret_cast<float*>(b);
  md->adam_m = reinterpret_cast<float*>(b + pb);
  md->adam_v = reinterpret_cast<float*>(b + 2 * pb);
  md->grad = reinterpret_cast<float*>(b + 3 * pb);
  md->frag = b + 4 * pb;
  *out = md;
  return PSI_OK;
}

psi_status model_destroy(psi_model* md) {
  delete md;
  return PSI_OK;
}

psi_status model_get(const psi_model* md, int what, float* out, uint32_t flags, hipStream_t st) {
  PSI_REQUIRE(md && out, "arguments must not be NULL");
  const float* src = what == 0 ? md->params : md->grad;
  const hipMemcpyKind kind = (flags & PSI_INPUT_HOST) ? hipMemcpyDeviceToHost
                                                      : hipMemcpyDeviceToDevice;
  PSI_HIP_CHECK(hipMemcpyAsync(out, src, 4 * size_t(kNParam), kind, st));
  if (flags & PSI_INPUT_HOST) PSI_HIP_CHECK(hipStreamSynchronize(st));
  return PSI_OK;
}

psi_status mpnn_workspace_size(const psi_operator* op, int training, size_t* bytes) {
  PSI_REQUIRE(op && bytes, "arguments must not be NULL");
  *bytes = mp_layout(op, training != 0, nullptr, nullptr);
  return PSI_OK;
}

psi_status mpnn_forward(psi_model* md, psi_operator* op, float* t_hat, double* s0, void* ws,
                        size_t ws_bytes, hipStream_t st) {
  psi_status r = check_pair(md, op);
  if (r != PSI_OK) return r;
  PSI_REQUIRE(ws, "workspace must not be NULL");
  const size_t need = mp_layout(op, false, nullptr, nullptr);
  if (ws_bytes < need) {
    set_error("workspace smaller than psi_mpnn_workspace_size reported");
    return PSI_ENOSPACE;
  }
  MpWs w{};
  mp_layout(op, false, &w, static_cast<char*>(ws));
  return forward<false>(md, op, w, t_hat, s0, nullptr, st);
}

psi_status mpnn_loss_backward(psi_model* md, psi_operator* op, const double* s_target,
                              double* loss, float* t_hat, void* ws, size_t ws_bytes,
                              hipStream_t st) {
  psi_status r = check_pair(md, op);
  if (r != PSI_OK) return r;
  PSI_REQUIRE(ws && s_target, "workspace and s_target must not be NULL");
  const size_t need = mp_layout(op, true, nullptr, nullptr);
  if (ws_bytes < need) {
    set_error("workspace smaller than psi_mpnn_workspace_size reported (training)");
    return PSI_ENOSPACE;
  }
  MpWs w{};
  mp_layout(op, true, &w, static_cast<char*>(ws));
  r = forward<true>(md, op, w, t_hat, nullptr, s_target, st);
  if (r != PSI_OK) return r;
  r = backward(md, op, w, s_target, st);
  if (r != PSI_OK) return r;
  if (loss) {
    MpCtrl h{};
    PSI_HIP_CHECK(hipMemcpyAsync(&h, w.ctrl, sizeof(MpCtrl), hipMemcpyDeviceToHost, st));
    PSI_HIP_CHECK(hipStreamSynchronize(st));
    *loss = h.loss;
  }
  return PSI_OK;
}

psi_status mpnn_adam_step(psi_model* md, double lr, double beta1, double beta2, double eps,
                          hipStream_t st) {
  PSI_REQUIRE(md, "model must not be NULL");
  PSI_REQUIRE(lr > 0.0 && beta1 >= 0.0 && beta1 < 1.0 && beta2 >= 0.0 && beta2 < 1.0 && eps > 0.0,
              "Adam needs lr > 0, beta1, beta2 in [0, 1), eps > 0");
  md->step += 1;
  const double c1 = 1.0 / (1.0 - std::pow(beta1, double(md->step)));
  const double c2 = 1.0 / (1.0 - std::pow(beta2, double(md->step)));
  hipLaunchKernelGGL(k_mp_adam, dim3(grid_for(kNParam)), dim3(kBlock), 0, st, md->params,
                     md->adam_m, md->adam_v, md->grad, kNParam, float(lr), float(beta1),
                     float(beta2), float(eps), float(c1), float(c2));
  PSI_HIP_CHECK(hipGetLastError());
  return refresh_frags(md, st);
}

}  // namespace psi
