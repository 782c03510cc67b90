// Training primitives shared by the learned surrogate and the PPO update:
// a BF16 MFMA GEMM (gfx950 v_mfma_f32_16x16x32_bf16, FP32 accumulation)
// with fused epilogues, a deterministic split-K path for the batch
// reductions of weight and bias gradients, and Adam.
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

#include "mlp.hpp"

namespace sgk {

__device__ __forceinline__ uint16_t bf16_bits(float x) {
  __bf16 b = (__bf16)x;  // round to nearest even
  return *reinterpret_cast<uint16_t*>(&b);
}
__device__ __forceinline__ float bf16_val(uint16_t u) { return __uint_as_float((uint32_t)u << 16); }

__device__ __forceinline__ float elu_f(float x) { return x > 0.f ? x : __expf(x) - 1.f; }
__device__ __forceinline__ float elu_grad_f(float z) { return z > 0.f ? 1.f : __expf(z); }

// Hidden-unit activations: ELU (surrogate), tanh (policy; the same formula
// as the rollout's forward pass, so both see the same activations).
enum { ACT_ELU = 0, ACT_TANH = 1 };
template <int ACT> __device__ __forceinline__ float act_f(float z) {
  return ACT == ACT_ELU ? elu_f(z) : tanh_fast(z);
}
template <int ACT> __device__ __forceinline__ float act_grad(float z) {
  if (ACT == ACT_ELU) return elu_grad_f(z);
  const float t = tanh_fast(z);
  return 1.f - t * t;
}

// C[m][n] = sum_k A(m, k) B(k, n) (+ epilogue), BF16 inputs, FP32
// accumulation. A(m, k) = A[AT ? k*lda + m : m*lda + k],
// B(k, n) = B[BT ? n*ldb + k : k*ldb + n]. Epilogues:
//   EPI_FWD_HIDDEN  z + bias -> C (FP32, if non-null), act(z) -> Cb (BF16)
//   EPI_FWD_OUT     z + bias -> C
//   EPI_PLAIN       z -> C
//   EPI_BWD_DX      z act'(Zp) -> C (if non-null) and Cb (backward through
//                   the unit); with colpart, the column sums of the block's
//                   64 rows as well (bias gradients without a second pass).
//                   Without Zp the pre-activations are recomputed from the
//                   forward's own operands (RA RB^T + rbias): the same MFMAs
//                   on the same BF16 data give the forward's FP32 values
//                   exactly, and for a narrow input layer this is cheaper
//                   than storing and re-reading them
//   EPI_PARTIAL     block z of the grid sums K in [z kchunk, (z+1) kchunk)
//                   and writes its partial to C + z M ldc (split-K; reduce
//                   with k_sum_two)
enum { EPI_FWD_HIDDEN = 0, EPI_FWD_OUT = 1, EPI_PLAIN = 2, EPI_BWD_DX = 3, EPI_PARTIAL = 4 };

struct GemmArgs {
  int M, N, K;
  const uint16_t* A;
  int lda;
  const uint16_t* B;
  int ldb;
  float* C;          // fp32 output [M][ldc] (split-K: [splits][M][ldc])
  int ldc;
  const float* bias; // [N] (forward)
  uint16_t* Cb;      // bf16 output [M][ldc] (act(z) forward, gradient backward)
  const float* Zp;   // pre-activations of the previous layer [M][ldc] (backward data)
  const uint16_t* RA;  // EPI_BWD_DX without Zp: the forward's A [M][rlda],
  int rlda;            // B [N][rldb] (row n = unit n), RK inputs, and bias
  const uint16_t* RB;
  int rldb, RK;
  const float* rbias;
  int kchunk;        // split-K chunk (multiple of 32)
  float* colpart;    // EPI_BWD_DX: per-block column sums of the result [gridDim.y][N] (may be null)
};

// One 64x64 output tile (block lin of a gx x gy x gz grid) of the GEMM g,
// for k_gemm and the grouped launch k_gemm_group.
template <int EPI, bool AT, bool BT, int ACT>
__device__ __forceinline__ void gemm_block(const GemmArgs& g, int lin, int gx, int gy, int gz) {
  // LDS tiles [row][k], 32 k + 8 pad; the four 8-k blocks of a row are
  // stored XOR-swizzled by (row / 8) mod 4, which spreads the transposing
  // stores below (one column of eight rows 8 apart per instruction) over
  // four banks instead of one
  __shared__ __align__(16) uint16_t As[64][40];
  __shared__ __align__(16) uint16_t Bs[64][40];
  auto swz = [](int row, int kb) { return (kb ^ ((row >> 3) & 3)) * 8; };
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  // Tile coordinates. Work-groups go to the 8 XCDs round-robin by linear id;
  // the remap hands each XCD a contiguous range of tiles (x fastest), so the
  // tiles that share a row slab (and a K-chunk) run on one XCD and re-read
  // it from that XCD's L2 instead of across the fabric.
  const int nblk = gx * gy * gz;
  if ((nblk & 7) == 0) lin = (lin & 7) * (nblk >> 3) + (lin >> 3);
  const int bx = lin % gx, by = (lin / gx) % gy, bz = lin / (gx * gy);
  const int m0 = by * 64, n0 = bx * 64;
  const int wm = (wave >> 1) * 32, wn = (wave & 1) * 32;
  const int gi = lane >> 4, li = lane & 15;
  int kbeg = 0, kend = g.K;
  float* C = g.C;
  if (EPI == EPI_PARTIAL) {
    kbeg = bz * g.kchunk;
    kend = min(g.K, kbeg + g.kchunk);
    C += (size_t)bz * g.M * g.ldc;
  }
  f32x4 acc[2][2];
#pragma unroll
  for (int a = 0; a < 2; ++a)
#pragma unroll
    for (int b = 0; b < 2; ++b) acc[a][b] = f32x4{0.f, 0.f, 0.f, 0.f};
  // Loaders. Contiguous-k operands (A row-major, B transposed): thread t
  // takes 8 consecutive k of row t / 4. Contiguous-m/n operands: thread t
  // takes 8 consecutive rows at k = t / 8. With 16-byte aligned rows each is
  // one vector load; otherwise (or at a ragged edge) element by element.
  // The next k-slice is fetched into registers while the current one is
  // multiplied (one slice in flight).
  const int lr = tid >> 2, lk = (tid & 3) * 8;
  const int tk = tid >> 3, tm = (tid & 7) * 8;
  const bool avec = (((uintptr_t)g.A) & 15) == 0 && (g.lda & 7) == 0;
  const bool bvec = (((uintptr_t)g.B) & 15) == 0 && (g.ldb & 7) == 0;
  auto fetch = [&](const uint16_t* X, int ld, bool vec, int rows, int r0, bool trans, int k0) -> uint4 {
    uint4 v = make_uint4(0, 0, 0, 0);
    if (!trans) {
      const int m = r0 + lr, k = k0 + lk;
      if (m < rows && k < kend) {
        if (vec && k + 8 <= kend) {
          v = *reinterpret_cast<const uint4*>(X + (size_t)m * ld + k);
        } else {
          uint16_t t[8];
#pragma unroll
          for (int s = 0; s < 8; ++s) t[s] = (k + s < kend) ? X[(size_t)m * ld + k + s] : 0;
          v = *reinterpret_cast<uint4*>(t);
        }
      }
    } else {
      const int k = k0 + tk, m = r0 + tm;
      if (k < kend && vec && m + 8 <= rows) {
        v = *reinterpret_cast<const uint4*>(X + (size_t)k * ld + m);
      } else {
        uint16_t t[8];
#pragma unroll
        for (int s = 0; s < 8; ++s) t[s] = (k < kend && m + s < rows) ? X[(size_t)k * ld + m + s] : 0;
        v = *reinterpret_cast<uint4*>(t);
      }
    }
    return v;
  };
  auto stash = [&](uint16_t (*S)[40], bool trans, const uint4& v) {
    if (!trans) {
      *reinterpret_cast<uint4*>(&S[lr][swz(lr, lk >> 3)]) = v;
    } else {
      uint16_t t[8];
      *reinterpret_cast<uint4*>(t) = v;
#pragma unroll
      for (int s = 0; s < 8; ++s) S[tm + s][swz(tm, tk >> 3) + (tk & 7)] = t[s];
    }
  };
  // The split-K weight gradients (long K loops, two blocks per CU) keep two
  // slices in flight: slice k0 is stashed while k0 + 32 is loading and
  // k0 + 64 is requested (a slice at or past kend loads as zeros). The
  // other GEMMs (K <= 256, eight blocks per CU) prefetch one.
  constexpr bool kPF2 = EPI == EPI_PARTIAL;
  uint4 ra = fetch(g.A, g.lda, avec, g.M, m0, AT, kbeg);
  uint4 rb = fetch(g.B, g.ldb, bvec, g.N, n0, !BT, kbeg);
  uint4 ra2 = make_uint4(0, 0, 0, 0), rb2 = make_uint4(0, 0, 0, 0);
  if (kPF2) {
    ra2 = fetch(g.A, g.lda, avec, g.M, m0, AT, kbeg + 32);
    rb2 = fetch(g.B, g.ldb, bvec, g.N, n0, !BT, kbeg + 32);
  }
  for (int k0 = kbeg; k0 < kend; k0 += 32) {
    stash(As, AT, ra);
    stash(Bs, !BT, rb);
    __syncthreads();
    if (kPF2) {
      ra = ra2;
      rb = rb2;
      if (k0 + 64 < kend) {
        ra2 = fetch(g.A, g.lda, avec, g.M, m0, AT, k0 + 64);
        rb2 = fetch(g.B, g.ldb, bvec, g.N, n0, !BT, k0 + 64);
      }
    } else if (k0 + 32 < kend) {
      ra = fetch(g.A, g.lda, avec, g.M, m0, AT, k0 + 32);
      rb = fetch(g.B, g.ldb, bvec, g.N, n0, !BT, k0 + 32);
    }
    bf16x8 af[2], bfr[2];
#pragma unroll
    for (int t = 0; t < 2; ++t) {
      af[t] = *reinterpret_cast<const bf16x8*>(&As[wm + 16 * t + li][swz(wm + 16 * t + li, gi)]);
      bfr[t] = *reinterpret_cast<const bf16x8*>(&Bs[wn + 16 * t + li][swz(wn + 16 * t + li, gi)]);
    }
#pragma unroll
    for (int a = 0; a < 2; ++a)
#pragma unroll
      for (int b = 0; b < 2; ++b) acc[a][b] = mfma16x16x32(af[a], bfr[b], acc[a][b]);
    __syncthreads();
  }
  f32x4 zr[2][2];  // EPI_BWD_DX without Zp: recomputed pre-activations
  if (EPI == EPI_BWD_DX && !g.Zp) {
#pragma unroll
    for (int a = 0; a < 2; ++a)
#pragma unroll
      for (int b = 0; b < 2; ++b) zr[a][b] = f32x4{0.f, 0.f, 0.f, 0.f};
    kend = g.RK;
    const bool rav = (((uintptr_t)g.RA) & 15) == 0 && (g.rlda & 7) == 0;
    const bool rbv = (((uintptr_t)g.RB) & 15) == 0 && (g.rldb & 7) == 0;
    for (int k0 = 0; k0 < g.RK; k0 += 32) {
      // the tiles are free: the main loop ended on a barrier
      stash(As, false, fetch(g.RA, g.rlda, rav, g.M, m0, false, k0));
      stash(Bs, false, fetch(g.RB, g.rldb, rbv, g.N, n0, false, k0));
      __syncthreads();
      bf16x8 af[2], bfr[2];
#pragma unroll
      for (int t = 0; t < 2; ++t) {
        af[t] = *reinterpret_cast<const bf16x8*>(&As[wm + 16 * t + li][swz(wm + 16 * t + li, gi)]);
        bfr[t] = *reinterpret_cast<const bf16x8*>(&Bs[wn + 16 * t + li][swz(wn + 16 * t + li, gi)]);
      }
#pragma unroll
      for (int a = 0; a < 2; ++a)
#pragma unroll
        for (int b = 0; b < 2; ++b) zr[a][b] = mfma16x16x32(af[a], bfr[b], zr[a][b]);
      __syncthreads();
    }
  }
  float cs[2] = {0.f, 0.f};  // EPI_BWD_DX: this lane's share of two column sums
#pragma unroll
  for (int a = 0; a < 2; ++a)
#pragma unroll
    for (int b = 0; b < 2; ++b)
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        const int m = m0 + wm + 16 * a + 4 * gi + r, n = n0 + wn + 16 * b + li;
        if (m >= g.M || n >= g.N) continue;
        const size_t i = (size_t)m * g.ldc + n;
        float z = acc[a][b][r];
        if (EPI == EPI_FWD_HIDDEN || EPI == EPI_FWD_OUT) z += g.bias[n];
        if (EPI == EPI_BWD_DX) {
          z *= act_grad<ACT>(g.Zp ? g.Zp[i] : zr[a][b][r] + g.rbias[n]);
          cs[b] += z;
        }
        if ((EPI != EPI_BWD_DX && EPI != EPI_FWD_HIDDEN) || C) C[i] = z;
        if (EPI == EPI_FWD_HIDDEN) g.Cb[i] = bf16_bits(act_f<ACT>(z));
        if (EPI == EPI_BWD_DX) g.Cb[i] = bf16_bits(z);
      }
  if (EPI == EPI_BWD_DX && g.colpart) {
    // columns n0 + wn + 16 b + li: add the four row groups of the wave, then
    // the two waves that share the columns, in a fixed order
    __shared__ float csum[2][2][32];
#pragma unroll
    for (int b = 0; b < 2; ++b) {
      cs[b] += __shfl_xor(cs[b], 16, 64);
      cs[b] += __shfl_xor(cs[b], 32, 64);
      if (gi == 0) csum[wm >> 5][wn >> 5][16 * b + li] = cs[b];
    }
    __syncthreads();
    if (tid < 64) {
      const int n = n0 + tid;
      if (n < g.N) g.colpart[(size_t)by * g.N + n] = csum[0][tid >> 5][tid & 31] + csum[1][tid >> 5][tid & 31];
    }
  }
}

// At most 64 VGPRs (8 waves per SIMD), so 8 blocks fit on a CU: the wide
// forward and data-gradient GEMMs launch 8 blocks per CU.
template <int EPI, bool AT, bool BT, int ACT>
__global__ void __launch_bounds__(256, 8) k_gemm(GemmArgs g) {
  gemm_block<EPI, AT, BT, ACT>(g, blockIdx.x + gridDim.x * (blockIdx.y + gridDim.y * blockIdx.z), gridDim.x,
                               gridDim.y, gridDim.z);
}

// Up to kMaxGemmGroup GEMMs of one kind in one launch: blocks [blk0[k],
// blk0[k + 1]) are GEMM k's grid gx[k] x gy[k] x gz[k] (each a multiple of
// 8 blocks where the XCD remap applies, so the groups' blocks keep their
// XCD assignment).
constexpr int kMaxGemmGroup = 4;
struct GemmGroup {
  GemmArgs g[kMaxGemmGroup];
  int gx[kMaxGemmGroup], gy[kMaxGemmGroup], gz[kMaxGemmGroup];
  int blk0[kMaxGemmGroup + 1];
  int count;
};
template <int EPI, bool AT, bool BT, int ACT>
__global__ void __launch_bounds__(256, 8) k_gemm_group(GemmGroup a) {
  int k = 0;
  while (k + 1 < a.count && (int)blockIdx.x >= a.blk0[k + 1]) ++k;
  gemm_block<EPI, AT, BT, ACT>(a.g[k], (int)blockIdx.x - a.blk0[k], a.gx[k], a.gy[k], a.gz[k]);
}

template <int EPI, bool AT, bool BT, int ACT>
static inline void launch_gemm(hipStream_t s, const GemmArgs& a, int splits = 1) {
  dim3 grid((a.N + 63) / 64, (a.M + 63) / 64, EPI == EPI_PARTIAL ? splits : 1);
  k_gemm<EPI, AT, BT, ACT><<<grid, 256, 0, s>>>(a);
}

// Split sums: out[i * ldo + j] = sum_z part[z * stride + i N + j] over
// `splits` slabs (stride 0: M N). A block covers 256 / G consecutive outputs
// with G thread groups, group g summing slabs g, g + G, ...; the G partial
// sums are then added in group order: deterministic for a given G. G (a
// power of two, 1..64) is chosen so each thread reads about eight slabs.
// Two independent jobs share one launch: blocks [0, blocks_a) reduce job
// a, the rest job b.
struct SumJob {
  const float* part;
  int splits, M, N;
  float* out;
  int ldo, stride;
  int groups;
};
static inline SumJob sum_job(const float* part, int splits, int M, int N, float* out, int ldo, int stride) {
  int g = 1;
  while (g < 64 && g * 8 < splits) g *= 2;
  return SumJob{part, splits, M, N, out, ldo, stride, g};
}
static inline int sum_job_blocks(const SumJob& j) {
  const int per = 256 / j.groups;
  return (j.M * j.N + per - 1) / per;
}
// Optional squared-norm partials of the summed values (the PPO update's
// gradient clip): an output at flat index [adj0, adj0 + adjn) of the vector
// at base is shifted by -adj before squaring (the entropy term on log_std),
// and block b of the launch writes its sum of squares (double, in a fixed
// order) to npart[b]. npart null: none.
struct SumNorm {
  const float* base;
  int adj0, adjn;
  float adj;
  double* npart;
};
// Block blk of job j (256 threads); returns this thread's squared
// contribution to the norm partial (0 unless nm.npart).
__device__ __forceinline__ double sum_block(const SumJob& j, int blk, const SumNorm& nm = SumNorm{}) {
  __shared__ float red[256];
  const int G = j.groups, per = 256 / G;
  const int slot = threadIdx.x % per, grp = threadIdx.x / per;
  const int o = blk * per + slot;
  const int MN = j.M * j.N;
  const size_t st = j.stride > 0 ? (size_t)j.stride : (size_t)MN;
  float s = 0.f;
  if (o < MN) {
    // this thread's slabs grp, grp + G, ... in order; eight loads in flight
    // at a time (the sum order is unchanged)
    int z = grp;
    for (; z + 7 * G < j.splits; z += 8 * G) {
      float v[8];
#pragma unroll
      for (int u = 0; u < 8; ++u) v[u] = j.part[(size_t)(z + u * G) * st + o];
#pragma unroll
      for (int u = 0; u < 8; ++u) s += v[u];
    }
    for (; z < j.splits; z += G) s += j.part[(size_t)z * st + o];
  }
  red[threadIdx.x] = s;
  __syncthreads();
  double sq = 0;
  if (grp == 0 && o < MN) {
    float t = 0.f;
    for (int k = 0; k < G; ++k) t += red[k * per + slot];
    float* dst = j.out + (size_t)(o / j.N) * j.ldo + o % j.N;
    *dst = t;
    if (nm.npart) {
      const long idx = dst - nm.base;
      const float v = idx >= nm.adj0 && idx < nm.adj0 + nm.adjn ? t - nm.adj : t;
      sq = (double)v * v;
    }
  }
  return sq;
}
static __global__ void __launch_bounds__(256) k_sum_two(SumJob a, int blocks_a, SumJob b) {
  if ((int)blockIdx.x < blocks_a) sum_block(a, blockIdx.x);
  else sum_block(b, blockIdx.x - blocks_a);
}
// Up to kMaxSumJobs independent jobs in one launch: blocks
// [blk0[k], blk0[k + 1]) reduce job k.
constexpr int kMaxSumJobs = 8;
struct SumJobs {
  SumJob j[kMaxSumJobs];
  int blk0[kMaxSumJobs + 1];
  int count;
  SumNorm nm;
};
static __global__ void __launch_bounds__(256) k_sum_jobs(SumJobs a) {
  int k = 0;
  while (k + 1 < a.count && (int)blockIdx.x >= a.blk0[k + 1]) ++k;
  double sq = sum_block(a.j[k], blockIdx.x - a.blk0[k], a.nm);
  if (a.nm.npart) {
    // the block's sum of squares: wave butterflies, then the four waves in order
    __shared__ double wsum[4];
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) sq += __shfl_xor(sq, o, 64);
    if ((threadIdx.x & 63) == 0) wsum[threadIdx.x >> 6] = sq;
    __syncthreads();
    if (threadIdx.x == 0) a.nm.npart[blockIdx.x] = (wsum[0] + wsum[1]) + (wsum[2] + wsum[3]);
  }
}
// Launches the jobs (with norm partials if nm.npart); returns the number of
// blocks (= norm partials written).
static inline int launch_sums(hipStream_t st, const SumJob* jobs, int n, const SumNorm& nm = SumNorm{}) {
  SumJobs a{};
  a.count = n;
  a.nm = nm;
  int b = 0;
  for (int k = 0; k < n; ++k) {
    a.j[k] = jobs[k];
    a.blk0[k] = b;
    b += sum_job_blocks(jobs[k]);
  }
  a.blk0[n] = b;
  k_sum_jobs<<<b, 256, 0, st>>>(a);
  return b;
}

// Split-K shape for a weight gradient: about 256 blocks over the output
// tiles, 512 (two per CU) for batches of 8192 rows and more, where a single
// block per CU would leave the long K loop waiting on memory latency; each
// block sums a chunk (multiple of 32) of the batch.
static inline int splits_for(int tiles, int K) {
  int s = (K >= 8192 ? 512 : 256) / (tiles > 0 ? tiles : 1);
  const int kmax = (K + 31) / 32;
  if (s > kmax) s = kmax;
  return s < 1 ? 1 : s;
}
static inline int chunk_for(int K, int splits) { return ((K + splits - 1) / splits + 31) / 32 * 32; }
// Floats of split-K partials the helper below may write: at most
// 512 / tiles splits of tiles x 64 x 64 outputs.
constexpr size_t kWeightGradWs = (size_t)512 * 64 * 64;

// dW [M][N] (leading dim ldo) = sum_b A(b, m) B(b, n) over a batch of K
// rows (A [K][lda], B [K][ldb], BF16): the split-K GEMM writes its partials
// to ws (kWeightGradWs floats); the returned job sums them into out.
template <int ACT>
static inline SumJob launch_weight_grad_partials(hipStream_t st, int M, int N, int K, const uint16_t* A, int lda,
                                                 const uint16_t* B, int ldb, float* out, int ldo, float* ws) {
  const int tiles = ((M + 63) / 64) * ((N + 63) / 64);
  const int S = splits_for(tiles, K);
  GemmArgs g{};
  g.M = M; g.N = N; g.K = K; g.A = A; g.lda = lda; g.B = B; g.ldb = ldb; g.C = ws; g.ldc = N;
  g.kchunk = chunk_for(K, S);
  const int S_eff = (K + g.kchunk - 1) / g.kchunk;
  launch_gemm<EPI_PARTIAL, true, false, ACT>(st, g, S_eff);
  return sum_job(ws, S_eff, M, N, out, ldo, 0);
}
// Several weight gradients (split-K partials) in one grouped launch: add()
// sets up one and returns the job that sums its partials; launch() runs
// them all.
template <int ACT> struct WeightGradGroup {
  GemmGroup grp{};
  int blocks = 0;
  SumJob add(int M, int N, int K, const uint16_t* A, int lda, const uint16_t* B, int ldb, float* out, int ldo,
             float* ws) {
    const int tiles = ((M + 63) / 64) * ((N + 63) / 64);
    const int S = splits_for(tiles, K);
    GemmArgs& g = grp.g[grp.count];
    g = GemmArgs{};
    g.M = M; g.N = N; g.K = K; g.A = A; g.lda = lda; g.B = B; g.ldb = ldb; g.C = ws; g.ldc = N;
    g.kchunk = chunk_for(K, S);
    const int S_eff = (K + g.kchunk - 1) / g.kchunk;
    grp.gx[grp.count] = (N + 63) / 64;
    grp.gy[grp.count] = (M + 63) / 64;
    grp.gz[grp.count] = S_eff;
    grp.blk0[grp.count] = blocks;
    blocks += grp.gx[grp.count] * grp.gy[grp.count] * S_eff;
    ++grp.count;
    return sum_job(ws, S_eff, M, N, out, ldo, 0);
  }
  void launch(hipStream_t st) {
    grp.blk0[grp.count] = blocks;
    if (grp.count) k_gemm_group<EPI_PARTIAL, true, false, ACT><<<blocks, 256, 0, st>>>(grp);
  }
};

// The same with the split sums launched at once, sharing their launch with
// `bias`, the reduction of a bias gradient's per-block partial rows.
template <int ACT>
static inline void launch_weight_grad(hipStream_t st, int M, int N, int K, const uint16_t* A, int lda,
                                      const uint16_t* B, int ldb, float* out, int ldo, float* ws,
                                      const SumJob& bias) {
  const SumJob w = launch_weight_grad_partials<ACT>(st, M, N, K, A, lda, B, ldb, out, ldo, ws);
  const int bw = sum_job_blocks(w);
  k_sum_two<<<bw + sum_job_blocks(bias), 256, 0, st>>>(w, bw, bias);
}

// out[c] = sum over `blocks` partial rows part[b][c] (row stride `stride`).
static inline SumJob partial_rows(const float* part, int blocks, int cols, int stride, float* out) {
  return sum_job(part, blocks, 1, cols, out, cols, stride);
}

// dst[i] = src[i] (a kernel rather than a copy node, so callers stay
// capturable).
static __global__ void __launch_bounds__(256) __attribute__((unused)) k_copy_f(const float* __restrict__ src, float* __restrict__ dst, int n) {
  const int i = blockIdx.x * 256 + threadIdx.x;
  if (i < n) dst[i] = src[i];
}

// Adam (Kingma & Ba) with bias correction c1 = 1 - beta1^t, c2 = 1 - beta2^t
// passed in, over up to kAdamSegs parameter arrays in one launch: segment
// k owns blocks [blk0_k, blk0_{k+1}); optional BF16 copy of the updated
// weights.
constexpr int kAdamSegs = 8;
struct AdamSeg {
  float* w;
  const float* g;
  float* m;
  float* v;
  uint16_t* wb;  // may be null
  int n, blk0;
};
struct AdamSegs {
  AdamSeg s[kAdamSegs];
  int count, blocks;
};
static inline void adam_add(AdamSegs& a, float* w, const float* g, float* m, float* v, uint16_t* wb, int n) {
  a.s[a.count] = AdamSeg{w, g, m, v, wb, n, a.blocks};
  a.blocks += (n + 255) / 256;
  a.count += 1;
}
static __global__ void __launch_bounds__(256) __attribute__((unused)) k_adam_segs(AdamSegs a, float lr, float b1, float b2, float eps, float c1,
                                                          float c2) {
  int k = 0;
  while (k + 1 < a.count && (int)blockIdx.x >= a.s[k + 1].blk0) ++k;
  const AdamSeg& sg = a.s[k];
  const int i = ((int)blockIdx.x - sg.blk0) * 256 + threadIdx.x;
  if (i >= sg.n) return;
  const float gi = sg.g[i];
  const float mi = b1 * sg.m[i] + (1.f - b1) * gi;
  const float vi = b2 * sg.v[i] + (1.f - b2) * gi * gi;
  sg.m[i] = mi;
  sg.v[i] = vi;
  const float wi = sg.w[i] - lr * (mi / c1) / (sqrtf(vi / c2) + eps);
  sg.w[i] = wi;
  if (sg.wb) sg.wb[i] = bf16_bits(wi);
}

static __global__ void __launch_bounds__(256) k_to_bf16(int n, const float* __restrict__ w,
                                                        uint16_t* __restrict__ wb) {
  const int i = blockIdx.x * 256 + threadIdx.x;
  if (i < n) wb[i] = bf16_bits(w[i]);
}

}  // namespace sgk
