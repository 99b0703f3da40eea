// Particle-particle ladder, mixed precision: split-bf16 with three products and FP32
// accumulation on bf16 MFMA (gfx950).
//
// Every FP64 operand x is split as x = hi + lo with hi = bf16(x) and lo = bf16(x - hi)
// (round to nearest even), and each product is formed as hi*hi + hi*lo + lo*hi
// (the lo*lo term, ~2^-16 relative, is dropped) with FP32 accumulation.  The
// algorithm is the one of the FP64 path (Sec. II.C, eq. pp-Ladder-0 with Scuseria's
// split): build W+- = (ac|bd) +- (ad|bc) tile by tile over the RI index, contract
// with packed tau+-, unpack the mirrored entries into the FP64 R.
//
// Layouts (bf16 stored as 16-bit words):
//   Bh/Bl [c][Q/32][a][32] factors in Q tiles of 32 (Q padded to 32): one 16-byte run
//                          holds the 8 consecutive Q a lane feeds to one MFMA, and the
//                          16 columns of one block read in a Q step are one 1 KB run
//   Th/Tl [slot/32][ij][32]       packed tau+- (or tau-) in tiles of 32 slots
//   Wh/Wl [slot/32][ab slot][32]  build output, already split, in tiles of 32 slots
// The contraction reads one tile (32 slots of a 256-row block, 16 KB per array) per k
// step as one contiguous run.
// Within a cd block pair the 256 slots are ordered so that the 16 (c, d) pairs one
// wave of the build owns are consecutive: slot = half*128 + wave*16 + i*4 + j with
// c = 8*half + 4*(wave>>2) + i, d = 4*(wave&3) + j.  A lane then stores its 16 results
// for one (a, b) as two 16-byte runs per array.
//
// MFMA v_mfma_f32_16x16x32_bf16 lane layout (measured): A[m][k] at lane m + 16*(k/8),
// element k%8; B[k][n] at lane n + 16*(k/8), element k%8; D[m][n] at lane
// n + 16*(m/4), element m%4.
#include <cstdint>

#include "ppl_shared.h"

namespace ri {
namespace ppl {

typedef __bf16 bf16x8_t __attribute__((ext_vector_type(8)));
typedef float f32x4_t __attribute__((ext_vector_type(4)));
typedef unsigned int u32x4_t __attribute__((ext_vector_type(4)));  // one 16-byte run

constexpr int QC = 32;  // RI functions per build step (= MFMA K)
constexpr int KB = 32;  // cd slots per contraction step (= MFMA K)
constexpr int CBM = 256;  // contraction tile rows
constexpr int CNT = 2 * CBM;  // contraction threads: CBM / 32 waves of 32 rows each

__host__ __device__ inline uint16_t bf16_bits(float f) {
  // round to nearest even (inputs are finite)
  uint32_t u = __builtin_bit_cast(uint32_t, f);
  u += 0x7FFFu + ((u >> 16) & 1u);
  return static_cast<uint16_t>(u >> 16);
}
__host__ __device__ inline float bf16_val(uint16_t h) {
  return __builtin_bit_cast(float, static_cast<uint32_t>(h) << 16);
}
__device__ inline void split_f64(double x, uint16_t& hi, uint16_t& lo) {
  hi = bf16_bits(static_cast<float>(x));
  lo = bf16_bits(static_cast<float>(x - static_cast<double>(bf16_val(hi))));
}
__device__ inline void split_f32(float x, uint16_t& hi, uint16_t& lo) {
  hi = bf16_bits(x);
  lo = bf16_bits(x - bf16_val(hi));
}

__device__ inline f32x4_t mfma_bf16(bf16x8_t a, bf16x8_t b, f32x4_t c) {
  return __builtin_amdgcn_mfma_f32_16x16x32_bf16(a, b, c, 0, 0, 0);
}
// c += a*b with both split: hi*lo + lo*hi first, then hi*hi
__device__ inline f32x4_t mfma3(bf16x8_t ah, bf16x8_t al, bf16x8_t bh, bf16x8_t bl, f32x4_t c) {
  c = mfma_bf16(ah, bl, c);
  c = mfma_bf16(al, bh, c);
  return mfma_bf16(ah, bh, c);
}

// LDS swizzles.  A ds_read_b128 is conflict-free when every group of 8 lanes
// (32 banks) -- or of 16 lanes (64 banks) -- covers distinct 16-byte bank groups.
// Build: a row e of 4 runs; run r of row e is stored at r ^ sw4(e).  Contraction:
// a row of 8 runs (hi/lo x 4); run q of row m is stored at q ^ sw8(m).
__host__ __device__ inline int sw4(int e) { return ((e >> 1) ^ (e >> 2)) & 3; }
__host__ __device__ inline int sw8(int m) { return (m ^ (m >> 3)) & 7; }

// slot (0..255) of a cd block pair -> (c_in, d_in)
__host__ __device__ inline void slot_cd(int slot, int& c_in, int& d_in) {
  const int h = slot >> 7, w = (slot >> 4) & 7, i = (slot >> 2) & 3, j = slot & 3;
  c_in = 8 * h + 4 * (w >> 2) + i;
  d_in = 4 * (w & 3) + j;
}

// ---------------------------------------------------------------- split relayout
// Bh/Bl[c][Q/32][a][32] from B[q][a][c] at B + q*qs + a*rs + c (zero padded).
// grid (Qp/32, vp/32, vp), block 256: one a, a 32 (Q) x 32 (c) tile
__global__ __launch_bounds__(256) void split_b_kernel(const double* __restrict__ B, long qs, long rs, int v,
                                                      int naux, int vp, int Qp, uint16_t* __restrict__ Bh,
                                                      uint16_t* __restrict__ Bl) {
  __shared__ double tile[32][33];
  const int q0 = blockIdx.x * 32, c0 = blockIdx.y * 32, a = blockIdx.z;
  const int tx = threadIdx.x & 31, ty = threadIdx.x >> 5;  // ty 0..7
  for (int r = 0; r < 4; ++r) {
    const int q = q0 + ty + 8 * r, c = c0 + tx;
    tile[ty + 8 * r][tx] = (q < naux && c < v && a < v) ? B[q * qs + a * rs + c] : 0.0;
  }
  __syncthreads();
  for (int r = 0; r < 4; ++r) {
    const int c = c0 + ty + 8 * r, q = q0 + tx;
    if (c >= vp) continue;  // vp is a multiple of 16, the tile of 32
    uint16_t hi, lo;
    split_f64(tile[tx][ty + 8 * r], hi, lo);
    const size_t idx = ((static_cast<size_t>(c) * (Qp / 32) + blockIdx.x) * vp + a) * 32 + tx;
    Bh[idx] = hi;
    Bl[idx] = lo;
  }
}

// ---------------------------------------------------------------- split pack
// Th/Tl[k/32][col][k%32] with k = pcd*256 + slot: sign > 0 tau+ (with the 1/2 on c == d)
// over i<=j columns, sign < 0 tau- over i<j columns; both from the pair-symmetric part of
// tau.  grid (nbp, ncol), block 256
__global__ __launch_bounds__(256) void pack_tau_bf16_kernel(const double* __restrict__ tau, int o, int v,
                                                            int sign, uint16_t* __restrict__ Th,
                                                            uint16_t* __restrict__ Tl) {
  int Cb, Db;
  tri_decode(blockIdx.x, Cb, Db);
  const int col = blockIdx.y, slot = threadIdx.x;
  int c_in, d_in;
  slot_cd(slot, c_in, d_in);
  const int c = Cb * TB + c_in, d = Db * TB + d_in;
  const int nreal = sign > 0 ? o * (o + 1) / 2 : o * (o - 1) / 2;
  double val = 0.0;
  if (d < v && (Cb < Db || c_in <= d_in) && (sign > 0 || c != d) && col < nreal) {
    int i, j;
    tri_decode(col, i, j);
    if (sign < 0) j += 1;
    const size_t vv = static_cast<size_t>(v) * v;
    const double* tij = tau + (static_cast<size_t>(i) * o + j) * vv;
    const double* tji = tau + (static_cast<size_t>(j) * o + i) * vv;
    const size_t cd = static_cast<size_t>(c) * v + d, dc = static_cast<size_t>(d) * v + c;
    const double x1 = tij[cd], x2 = tij[dc], x3 = tji[cd], x4 = tji[dc];
    if (sign > 0) {
      val = 0.25 * ((x1 + x4) + (x2 + x3));
      if (c == d) val *= 0.5;
    } else {
      val = 0.25 * ((x1 + x4) - (x2 + x3));
    }
  }
  uint16_t hi, lo;
  split_f64(val, hi, lo);
  const size_t k = static_cast<size_t>(blockIdx.x) * 256 + slot;
  const size_t idx = (k / KB * gridDim.y + col) * KB + k % KB;
  Th[idx] = hi;
  Tl[idx] = lo;
}

// ---------------------------------------------------------------- build
// Diagonal ab block pairs (a and b in one block).  One workgroup = the block pair x one
// half of a cd block pair: the 8 c of half h of block Cb by all 16 d of block Db.  Eight
// waves; wave w owns c in 8h + 4(w>>2) + 0..3 and d in 4(w&3) + 0..3.  A Q step stages
// 24 factor rows (8 c, 16 d).  LDS: a ring of three 48 KB slots.  A step occupies two
// slots (factor rows 0-11 in the first, 12-23 in the second); while step s is computed,
// the first half of step s + 1 is written into the third slot, and its second half
// into step s's first slot once every wave has read it.  Each slot holds 16-byte runs
// [x 12][hl 2][e 32][run 4], the run index XOR-swizzled with sw4(e) so that the lanes of
// one ds_read_b128 hit distinct banks.  In a diagonal pair the (ad|bc) tile is the
// transpose of the (ac|bd) tile: only the latter is built, and the epilogue reads it
// back through LDS.  blockIdx.y counts the diagonal pairs from block Ab = diag_y0; the
// launch covers cd block pairs pcd0 .. nbp-1.
// grid ((nbp - pcd0)*2, diagonal pairs), block 512
constexpr int SLOT = 12 * 2 * 32 * 4;  // runs per LDS slot (48 KB)
__device__ __forceinline__ void build_diag_body(const uint16_t* __restrict__ Bh, const uint16_t* __restrict__ Bl,
                                                  int Qp, int vp, long slab0, long wts, int want_minus, int diag_y0,
                                                  long pcd0, uint16_t* __restrict__ Wph, uint16_t* __restrict__ Wpl,
                                                  uint16_t* __restrict__ Wmh, uint16_t* __restrict__ Wml) {
  __shared__ u32x4_t lds[3 * SLOT];
  static_assert(3 * SLOT * 4 >= 8 * 16 * 256, "the ring holds the transposed tiles");
  const int half = blockIdx.x & 1;
  const long pcd = pcd0 + (blockIdx.x >> 1);
  int Cb, Db, Ab, Bb;
  tri_decode(pcd, Cb, Db);
  Ab = Bb = diag_y0 + static_cast<int>(blockIdx.y);
  const long pab_loc = static_cast<long>(Ab) * (Ab + 3) / 2 - slab0;
  const int c_base = Cb * TB + half * 8;
  const int d_base = Db * TB;
  const int t = threadIdx.x, w = t >> 6, lane = t & 63;

  // staging: run r (0..11) of a thread is run id = t + 512*r of the step, i.e. factor
  // row x = 2r + (t >> 8) (x < 8: c rows, else d rows) with the thread's own
  // (hl, e, run); runs 0-5 go to the step's first slot, 6-11 to its second.  The hi/lo
  // array and the row parity are uniform over a wave, so the loads are buffer loads
  // from two wave-uniform resources with one per-lane byte offset and a uniform offset
  // per run and Q step.
  const int wave = __builtin_amdgcn_readfirstlane(t >> 6);
  const int hl_w = (wave >> 1) & 1, xt = wave >> 2, e_t = (t >> 2) & 31, run_t = t & 3;
  const int ag = e_t < 16 ? Ab * TB + e_t : Bb * TB + (e_t - 16);
  const uint16_t* src = hl_w ? Bl : Bh;
  const size_t xs = static_cast<size_t>(vp) * Qp;  // elements from one factor row x to the next
  const __amdgpu_buffer_rsrc_t rc = __builtin_amdgcn_make_buffer_rsrc(
      const_cast<uint16_t*>(src + static_cast<size_t>(c_base + xt) * xs), 0, -1, 0x00020000);
  const __amdgpu_buffer_rsrc_t rd = __builtin_amdgcn_make_buffer_rsrc(
      const_cast<uint16_t*>(src + static_cast<size_t>(d_base + xt) * xs), 0, -1, 0x00020000);
  const int voff = (ag * 32 + run_t * 8) * 2;  // bytes within the Q tile
  const int xsb2 = static_cast<int>(xs * 4);  // bytes for two factor rows
  // LDS run of staging run r within its slot: x' = x mod 12 = 2(r mod 6) + xt
  const int l0 = xt * 256 + (hl_w * 32 + e_t) * 4 + (run_t ^ sw4(e_t));  // + 512 per run
  auto gload = [&](u32x4_t* dst, int h2, int step) {  // runs 6*h2 .. 6*h2 + 5
    const int qb = step * vp * QC * 2;  // bytes: one Q tile of vp columns per step
#pragma unroll
    for (int k = 0; k < 6; ++k) {
      const int r = 6 * h2 + k;
      dst[k] = __builtin_bit_cast(u32x4_t, r < 4 ? __builtin_amdgcn_raw_buffer_load_b128(rc, voff, r * xsb2 + qb, 0)
                                                 : __builtin_amdgcn_raw_buffer_load_b128(rd, voff, (r - 4) * xsb2 + qb, 0));
    }
  };
  auto lstore = [&](const u32x4_t* sv, int slot) {
#pragma unroll
    for (int k = 0; k < 6; ++k) lds[slot * SLOT + l0 + 512 * k] = sv[k];
  };
  // fragment addresses (run indices) for this lane
  const int fe = lane & 15, frun = lane >> 4;
  const int fsw = frun ^ sw4(fe);  // same swizzle for e and e + 16 (sw4 reads bits 1..3)
  const int xc0 = (w >> 2) * 4, xd0 = 8 + (w & 3) * 4;

  f32x4_t o1[4][4], o2[4][4];
#pragma unroll
  for (int i = 0; i < 4; ++i)
#pragma unroll
    for (int j = 0; j < 4; ++j) {
      o1[i][j] = f32x4_t{0.f, 0.f, 0.f, 0.f};
      o2[i][j] = f32x4_t{0.f, 0.f, 0.f, 0.f};
    }

  const int nsteps = Qp / QC;
  // in a diagonal cd block pair the slots with c > d carry zero amplitudes: a wave whose
  // 4 x 4 pairs all have c > d skips its products (uniform over the wave)
  const bool zero_w = Cb == Db && half == 1 && (w & 3) < 2;
  {
    // one Q step from the slots (s0: rows 0-11, s1: rows 12-23) into the accumulators
    auto compute = [&](int s0, int s1) {
      auto frag = [&](int x, int hl, int e_off) -> bf16x8_t {
        const int base = x < 12 ? s0 * SLOT : s1 * SLOT;
        const int xx = x < 12 ? x : x - 12;
        const u32x4_t v = lds[base + ((xx * 2 + hl) * 32 + e_off + fe) * 4 + fsw];
        return __builtin_bit_cast(bf16x8_t, v);
      };
      {  // (ac|bd): c fragments of the a rows with d fragments of the b rows
        bf16x8_t ac[4][2];
#pragma unroll
        for (int i = 0; i < 4; ++i)
#pragma unroll
          for (int hl = 0; hl < 2; ++hl) ac[i][hl] = frag(xc0 + i, hl, 0);
#pragma unroll
        for (int j = 0; j < 4; ++j) {
          const bf16x8_t bdh = frag(xd0 + j, 0, 16), bdl = frag(xd0 + j, 1, 16);
#pragma unroll
          for (int i = 0; i < 4; ++i) o1[i][j] = mfma3(ac[i][0], ac[i][1], bdh, bdl, o1[i][j]);
        }
      }
    };
    u32x4_t sa[6], sb[6];  // first and second half of the next step
    gload(sa, 0, 0);
    gload(sb, 1, 0);
    lstore(sa, 0);
    lstore(sb, 1);
    if (nsteps > 1) {
      gload(sa, 0, 1);
      gload(sb, 1, 1);
    }
    __syncthreads();
    int s0 = 0;  // slot of the current step's first half; its second half is s0 + 1 mod 3
    for (int st = 0; st < nsteps; ++st) {
      const int s1 = s0 == 2 ? 0 : s0 + 1, sf = s1 == 2 ? 0 : s1 + 1;
      const bool more = st + 1 < nsteps;
      if (more) {
        lstore(sa, sf);  // first half of step st + 1 into the free slot
        if (st + 2 < nsteps) gload(sa, 0, st + 2);
      }
      if (!zero_w) compute(s0, s1);
      __syncthreads();  // every wave has read slot s0
      if (more) {
        lstore(sb, s0);  // second half of step st + 1
        if (st + 2 < nsteps) gload(sb, 1, st + 2);
        __syncthreads();
      }
      s0 = sf;
    }
  }

  {
    // (ad|bc)[a][b] = (ac|bd)[b][a]: each wave stores its sixteen (ac|bd) tiles in its
    // own 16 KB of the ring, element (a, b) at a*16 + (b ^ a), and reads them back
    // transposed (the loop ended with every wave past its last fragment read)
    float* tw = reinterpret_cast<float*>(lds) + w * (16 * 256);
#pragma unroll
    for (int i = 0; i < 4; ++i)
#pragma unroll
      for (int j = 0; j < 4; ++j)
#pragma unroll
        for (int r = 0; r < 4; ++r) {
          const int a_in = 4 * (lane >> 4) + r, b_in = lane & 15;
          tw[(i * 4 + j) * 256 + a_in * 16 + (b_in ^ a_in)] = o1[i][j][r];
        }
    __syncthreads();
#pragma unroll
    for (int i = 0; i < 4; ++i)
#pragma unroll
      for (int j = 0; j < 4; ++j)
#pragma unroll
        for (int r = 0; r < 4; ++r) {
          const int a_in = 4 * (lane >> 4) + r, b_in = lane & 15;
          o2[i][j][r] = tw[(i * 4 + j) * 256 + b_in * 16 + (a_in ^ b_in)];
        }
  }

  // epilogue: lane holds (a_in = 4*(lane>>4) + r, b_in = lane&15) for the wave's 16
  // slots, stored as two 16-byte runs per array
  const size_t slot0 = static_cast<size_t>(pcd) * 256 + half * 128 + w * 16;
#pragma unroll
  for (int r = 0; r < 4; ++r) {
    const int a_in = 4 * (lane >> 4) + r, b_in = lane & 15;
    const size_t row = static_cast<size_t>(pab_loc) * 256 + a_in * 16 + b_in;
#pragma unroll
    for (int hh = 0; hh < 2; ++hh) {
      uint16_t ph[8], pl[8], mh[8], ml[8];
#pragma unroll
      for (int i = 0; i < 2; ++i)
#pragma unroll
        for (int j = 0; j < 4; ++j) {
          const float v1 = o1[2 * hh + i][j][r], v2 = o2[2 * hh + i][j][r];
          split_f32(v1 + v2, ph[i * 4 + j], pl[i * 4 + j]);
          split_f32(v1 - v2, mh[i * 4 + j], ml[i * 4 + j]);
        }
      u32x4_t h, l;
#pragma unroll
      for (int k = 0; k < 4; ++k) {
        h[k] = static_cast<uint32_t>(ph[2 * k]) | (static_cast<uint32_t>(ph[2 * k + 1]) << 16);
        l[k] = static_cast<uint32_t>(pl[2 * k]) | (static_cast<uint32_t>(pl[2 * k + 1]) << 16);
      }
      const size_t k = slot0 + 8 * hh;
      const size_t at = k / KB * wts + row * KB + k % KB;
      *reinterpret_cast<u32x4_t*>(Wph + at) = h;
      *reinterpret_cast<u32x4_t*>(Wpl + at) = l;
      if (want_minus) {
#pragma unroll
        for (int k = 0; k < 4; ++k) {
          h[k] = static_cast<uint32_t>(mh[2 * k]) | (static_cast<uint32_t>(mh[2 * k + 1]) << 16);
          l[k] = static_cast<uint32_t>(ml[2 * k]) | (static_cast<uint32_t>(ml[2 * k + 1]) << 16);
        }
        *reinterpret_cast<u32x4_t*>(Wmh + at) = h;
        *reinterpret_cast<u32x4_t*>(Wml + at) = l;
      }
    }
  }
}
// Off-diagonal ab block pairs, one integral per wave.  The workgroup covers the same
// tile as above (ab block pair x half h of cd block pair: 8 c by 16 d, the same 24
// staged factor rows per Q step), but wave w computes only one of the two integrals,
// g = w >> 2 (0: (ac|bd), 1: (ad|bc)), for 4 c by 8 d: c = 8h + 4(q >> 1) + i,
// d = 8(q & 1) + j with q = w & 3.  Per Q step a wave then reads 24 fragments for 96
// MFMAs instead of 32 (both integrals for 4 x 4 pairs), with the same 128 accumulator
// registers.  Both integrals run one instruction stream: a wave's first operand is its
// c fragment, its second the d fragment; the (ac|bd) waves read the c rows at the a
// columns and the d rows at the b columns and so hold element (a, b) of each tile,
// the (ad|bc) waves read the c rows at the b columns and the d rows at the a columns
// and hold the transposed tile, element (b, a).  After the Q loop the (ad|bc) waves
// pass their tiles through LDS, transposed back on the way, and the (ac|bd) waves
// write W+- for their 32 pairs into the slots of the slot order above.  The (ad|bc)
// products of (a, b) are then those of the (ac|bd) tile of (b, a) in the same order,
// so where both exist for one (a, b, c, d) they agree bit for bit.  The launch covers
// cd block pairs pcd0 .. nbp-1; diagonal ab block pairs exit (the diagonal kernel
// builds them).  Block 512.
// Workgroup order: the workgroups of one ab block pair and a square tile of T x T cd
// block pairs (c blocks by d blocks, both halves: 2T^2 workgroups, the tiles counted
// triangularly from the tile row of pcd0's d block) form a group; consecutive groups
// (cd tiles fastest, then ga ab block pairs) go round-robin to the eight XCDs in
// dispatch order (workgroup id mod 8), so the workgroups one XCD runs together read
// the factor rows of 2T blocks.  One-dimensional grid of 8 * ceil(groups / 8) * ga *
// 2T^2 workgroups; false for those that cover no pair (c block > d block, cd pairs
// before pcd0, the padding).
__device__ inline bool group_tile(int nb, long pcd0, long npairs, int ga, int T, long& pab, long& pcd, int& half) {
  const long GT = 2L * T * T;
  const long L = blockIdx.x, x = L & 7, p = L >> 3, G = static_cast<long>(ga) * GT;
  const long gi = (p / G) * 8 + x, r = p % G;
  int C0, D0;
  tri_decode(pcd0, C0, D0);
  const long nT = (nb + T - 1) / T, k0 = D0 / T, t0 = k0 * (k0 + 1) / 2;
  const long ntile = nT * (nT + 1) / 2 - t0, nga = (npairs + ga - 1) / ga;
  if (gi >= ntile * nga) return false;
  pab = (gi / ntile) * ga + r / GT;
  int tj, tk;
  tri_decode(t0 + gi % ntile, tj, tk);
  const int rr = static_cast<int>(r % GT);
  half = rr & 1;
  const int C = tj * T + (rr >> 1) % T, D = tk * T + (rr >> 1) / T;
  if (pab >= npairs || C > D || D >= nb) return false;
  pcd = static_cast<long>(D) * (D + 1) / 2 + C;
  return pcd >= pcd0;
}

__device__ __forceinline__ void build_split_body(const uint16_t* __restrict__ Bh, const uint16_t* __restrict__ Bl,
                                                 int Qp, int vp, long slab0, long wts, int want_minus, long pcd0,
                                                 long npairs, int ga, int gt,
                                                 uint16_t* __restrict__ Wph, uint16_t* __restrict__ Wpl,
                                                 uint16_t* __restrict__ Wmh, uint16_t* __restrict__ Wml) {
  __shared__ u32x4_t lds[3 * SLOT];
  static_assert(3 * SLOT * 16 >= 4 * 32 * 4 * 64 * 4, "the ring holds the exchanged (ad|bc) tiles");
  long pab_loc, pcd;
  int half;
  if (!group_tile(vp / TB, pcd0, npairs, ga, gt, pab_loc, pcd, half)) return;
  int Cb, Db, Ab, Bb;
  tri_decode(pcd, Cb, Db);
  tri_decode(slab0 + pab_loc, Ab, Bb);
  if (Ab == Bb) return;  // built by the diagonal launch (uniform over the workgroup)
  const int c_base = Cb * TB + half * 8;
  const int d_base = Db * TB;
  const int t = threadIdx.x, w = t >> 6, lane = t & 63;

  // staging: as in build_diag_body
  const int wave = __builtin_amdgcn_readfirstlane(t >> 6);
  const int hl_w = (wave >> 1) & 1, xt = wave >> 2, e_t = (t >> 2) & 31, run_t = t & 3;
  const int ag = e_t < 16 ? Ab * TB + e_t : Bb * TB + (e_t - 16);
  const uint16_t* src = hl_w ? Bl : Bh;
  const size_t xs = static_cast<size_t>(vp) * Qp;
  const __amdgpu_buffer_rsrc_t rc = __builtin_amdgcn_make_buffer_rsrc(
      const_cast<uint16_t*>(src + static_cast<size_t>(c_base + xt) * xs), 0, -1, 0x00020000);
  const __amdgpu_buffer_rsrc_t rd = __builtin_amdgcn_make_buffer_rsrc(
      const_cast<uint16_t*>(src + static_cast<size_t>(d_base + xt) * xs), 0, -1, 0x00020000);
  const int voff = (ag * 32 + run_t * 8) * 2;
  const int xsb2 = static_cast<int>(xs * 4);
  const int l0 = xt * 256 + (hl_w * 32 + e_t) * 4 + (run_t ^ sw4(e_t));
  auto gload = [&](u32x4_t* dst, int h2, int step) {
    const int qb = step * vp * QC * 2;
#pragma unroll
    for (int k = 0; k < 6; ++k) {
      const int r = 6 * h2 + k;
      dst[k] = __builtin_bit_cast(u32x4_t, r < 4 ? __builtin_amdgcn_raw_buffer_load_b128(rc, voff, r * xsb2 + qb, 0)
                                                 : __builtin_amdgcn_raw_buffer_load_b128(rd, voff, (r - 4) * xsb2 + qb, 0));
    }
  };
  auto lstore = [&](const u32x4_t* sv, int slot) {
#pragma unroll
    for (int k = 0; k < 6; ++k) lds[slot * SLOT + l0 + 512 * k] = sv[k];
  };
  const int fe = lane & 15, frun = lane >> 4;
  const int fsw = frun ^ sw4(fe);
  const int g = w >> 2, q = w & 3;
  const int xc0 = (q >> 1) * 4, xd0 = 8 + (q & 1) * 8;
  // (ac|bd) reads the c rows at the a columns (e 0..15) and the d rows at the b columns
  // (e 16..31); (ad|bc) the c rows at the b columns and the d rows at the a columns
  const int ec = g ? 16 : 0, ed = g ? 0 : 16;

  f32x4_t o[4][8];
#pragma unroll
  for (int i = 0; i < 4; ++i)
#pragma unroll
    for (int j = 0; j < 8; ++j) o[i][j] = f32x4_t{0.f, 0.f, 0.f, 0.f};

  const int nsteps = Qp / QC;
  // in a diagonal cd block pair the slots with c > d carry zero amplitudes: with c in the upper half and d in the
  // lower one every pair of the wave has c > d.  Such a wave runs the same products (a
  // branch around them costs the loop its schedule) and stores zeros.
  const bool zero_w = Cb == Db && half == 1 && (q & 1) == 0;
  {
    auto compute = [&](int s0, int s1) {
      auto frag = [&](int x, int hl, int e_off) -> bf16x8_t {
        const int base = x < 12 ? s0 * SLOT : s1 * SLOT;
        const int xx = x < 12 ? x : x - 12;
        const u32x4_t v = lds[base + ((xx * 2 + hl) * 32 + e_off + fe) * 4 + fsw];
        return __builtin_bit_cast(bf16x8_t, v);
      };
      bf16x8_t cf[4][2];
#pragma unroll
      for (int i = 0; i < 4; ++i)
#pragma unroll
        for (int hl = 0; hl < 2; ++hl) cf[i][hl] = frag(xc0 + i, hl, ec);
#pragma unroll
      for (int j = 0; j < 8; ++j) {
        const bf16x8_t dh = frag(xd0 + j, 0, ed), dl = frag(xd0 + j, 1, ed);
#pragma unroll
        for (int i = 0; i < 4; ++i) o[i][j] = mfma3(cf[i][0], cf[i][1], dh, dl, o[i][j]);
      }
      // issue order: the c fragments and the first d pair, then per d the 12 products
      // with the next d pair's reads ahead of them
      __builtin_amdgcn_sched_group_barrier(0x100, 12, 0);
#pragma unroll
      for (int j = 0; j < 7; ++j) {
        __builtin_amdgcn_sched_group_barrier(0x008, 12, 0);
        __builtin_amdgcn_sched_group_barrier(0x100, 2, 0);
      }
      __builtin_amdgcn_sched_group_barrier(0x008, 12, 0);
    };
    u32x4_t sa[6], sb[6];
    gload(sa, 0, 0);
    gload(sb, 1, 0);
    lstore(sa, 0);
    lstore(sb, 1);
    if (nsteps > 1) {
      gload(sa, 0, 1);
      gload(sb, 1, 1);
    }
    __syncthreads();
    int s0 = 0;
    for (int st = 0; st < nsteps; ++st) {
      const int s1 = s0 == 2 ? 0 : s0 + 1, sf = s1 == 2 ? 0 : s1 + 1;
      const bool more = st + 1 < nsteps;
      if (more) {
        lstore(sa, sf);
        if (st + 2 < nsteps) gload(sa, 0, st + 2);
      }
      compute(s0, s1);
      __syncthreads();
      if (more) {
        lstore(sb, s0);
        if (st + 2 < nsteps) gload(sb, 1, st + 2);
        __syncthreads();
      }
      s0 = sf;
    }
  }

  // exchange: the (ad|bc) wave q stores its tiles at [q][i][j][r][lane] (floats), the
  // (ac|bd) wave q reads them back in the same order (the loop ended with a barrier
  // after every wave's last fragment read)
  float* xb = reinterpret_cast<float*>(lds);
  const int m_l = 4 * (lane >> 4), n_l = lane & 15;  // a lane holds element (m_l + r, n_l)
  if (g == 1) {
    // element (m, n) of tile (q, i, j) at float m*16 + 4((n >> 2) ^ ((m >> 2) & 3)) + (n & 3)
    // of the tile's 1 KB: conflict-free stores here and loads below
#pragma unroll
    for (int i = 0; i < 4; ++i)
#pragma unroll
      for (int j = 0; j < 8; ++j)
#pragma unroll
        for (int r = 0; r < 4; ++r) {
          const int m = m_l + r;
          xb[((q * 4 + i) * 8 + j) * 256 + m * 16 + 4 * ((n_l >> 2) ^ ((m >> 2) & 3)) + (n_l & 3)] = o[i][j][r];
        }
  }
  __syncthreads();
  if (g == 1) return;
  // (ad|bc) at this lane's (a, b) = (m_l + r, n_l): element (n_l, m_l + r) of the stored tile
  auto xval = [&](int i, int j, int r) -> float {
    const int n = m_l + r;
    return xb[((q * 4 + i) * 8 + j) * 256 + n_l * 16 + 4 * ((n >> 2) ^ ((n_l >> 2) & 3)) + (n & 3)];
  };

  // epilogue: (c, d) = (8h + 4(q>>1) + i, 8(q&1) + j) sits in slot
  // h*128 + ow*16 + i*4 + (j & 3) with ow = 4(q>>1) + 2(q&1) + (j>>2) (the slot order of
  // the pack); a lane holds (a_in = 4(lane>>4) + r, b_in = lane&15) and stores, per ow
  // and pair of i, one 16-byte run per array
#pragma unroll
  for (int r = 0; r < 4; ++r) {
    const int a_in = 4 * (lane >> 4) + r, b_in = lane & 15;
    const size_t row = static_cast<size_t>(pab_loc) * 256 + a_in * 16 + b_in;
#pragma unroll
    for (int jb = 0; jb < 2; ++jb) {
      const int ow = 4 * (q >> 1) + 2 * (q & 1) + jb;
      const size_t slot0 = static_cast<size_t>(pcd) * 256 + half * 128 + ow * 16;
#pragma unroll
      for (int hh = 0; hh < 2; ++hh) {
        uint16_t ph[8], pl[8], mh[8], ml[8];
#pragma unroll
        for (int i2 = 0; i2 < 2; ++i2)
#pragma unroll
          for (int j2 = 0; j2 < 4; ++j2) {
            const int i = 2 * hh + i2, j = 4 * jb + j2;
            const float v1 = zero_w ? 0.f : o[i][j][r], v2 = zero_w ? 0.f : xval(i, j, r);
            split_f32(v1 + v2, ph[i2 * 4 + j2], pl[i2 * 4 + j2]);
            split_f32(v1 - v2, mh[i2 * 4 + j2], ml[i2 * 4 + j2]);
          }
        u32x4_t h, l;
#pragma unroll
        for (int k = 0; k < 4; ++k) {
          h[k] = static_cast<uint32_t>(ph[2 * k]) | (static_cast<uint32_t>(ph[2 * k + 1]) << 16);
          l[k] = static_cast<uint32_t>(pl[2 * k]) | (static_cast<uint32_t>(pl[2 * k + 1]) << 16);
        }
        const size_t k = slot0 + 8 * hh;
        const size_t at = k / KB * wts + row * KB + k % KB;
        *reinterpret_cast<u32x4_t*>(Wph + at) = h;
        *reinterpret_cast<u32x4_t*>(Wpl + at) = l;
        if (want_minus) {
#pragma unroll
          for (int k = 0; k < 4; ++k) {
            h[k] = static_cast<uint32_t>(mh[2 * k]) | (static_cast<uint32_t>(mh[2 * k + 1]) << 16);
            l[k] = static_cast<uint32_t>(ml[2 * k]) | (static_cast<uint32_t>(ml[2 * k + 1]) << 16);
          }
          *reinterpret_cast<u32x4_t*>(Wmh + at) = h;
          *reinterpret_cast<u32x4_t*>(Wml + at) = l;
        }
      }
    }
  }
}
__global__ __launch_bounds__(512) void build_w_bf16x3(const uint16_t* __restrict__ Bh, const uint16_t* __restrict__ Bl,
                                                      int Qp, int vp, long slab0, long wts, int want_minus, long pcd0,
                                                      long npairs, int ga, int gt, uint16_t* __restrict__ Wph,
                                                      uint16_t* __restrict__ Wpl, uint16_t* __restrict__ Wmh,
                                                      uint16_t* __restrict__ Wml) {
  build_split_body(Bh, Bl, Qp, vp, slab0, wts, want_minus, pcd0, npairs, ga, gt, Wph, Wpl, Wmh, Wml);
}
__global__ __launch_bounds__(512) void build_w_bf16x3_diag(const uint16_t* __restrict__ Bh,
                                                           const uint16_t* __restrict__ Bl, int Qp, int vp, long slab0,
                                                           long wts, int want_minus, int diag_y0, long pcd0,
                                                           uint16_t* __restrict__ Wph, uint16_t* __restrict__ Wpl,
                                                           uint16_t* __restrict__ Wmh, uint16_t* __restrict__ Wml) {
  build_diag_body(Bh, Bl, Qp, vp, slab0, wts, want_minus, diag_y0, pcd0, Wph, Wpl, Wmh, Wml);
}

// ---------------------------------------------------------------- contract
// C[m][n] (+)= sum_k W[m][k] T[n][k], both split and stored in tiles of KB k: element
// (m, k) of W at (k / KB) * lda + m * KB + k % KB (lda: elements from one tile to the
// next), of T likewise with ldb; tile
// CBM (m) x 16*NTW (n); CBM/32 waves, wave w owns rows 32w..32w+31 (two m tiles) and all
// columns.  LDS holds 16-byte runs [row][8 runs: hl 2 x run 4], run index XOR-swizzled
// with sw8(row).  The k range may be split over grid.z: split z sums k in
// [z*kz, min(K, (z+1)*kz)) into C + z*zs.  accum adds into C instead of writing it.
// grid (ncol/(16*NTW), rows/CBM, splits), block CNT
template <int NTW>
__global__ __launch_bounds__(CNT) void contract_bf16x3(const uint16_t* __restrict__ Wh, const uint16_t* __restrict__ Wl,
                                                       long lda, const uint16_t* __restrict__ Th,
                                                       const uint16_t* __restrict__ Tl, long ldb, long K, int ncol,
                                                       float* __restrict__ C, long kz, long zs, int accum) {
  constexpr int BN = 16 * NTW;
  constexpr int ARUNS = CBM * 2 * 4, BRUNS = BN * 2 * 4;
  __shared__ u32x4_t sA[2 * ARUNS];
  __shared__ u32x4_t sB[2 * BRUNS];
  unsigned tx, ty;
  xcd_tile(tx, ty);
  const long n0 = static_cast<long>(tx) * BN, m0 = static_cast<long>(ty) * CBM;
  const int t = threadIdx.x, w = t >> 6, lane = t & 63;
  // this split's k range (every split holds at least one step)
  const long k_lo = blockIdx.z * kz;
  const long k_len = (K < k_lo + kz ? K : k_lo + kz) - k_lo;
  C += blockIdx.z * zs;

  // staging: A 8*CBM runs (4 per thread), B 8*BN runs (BPER per thread, the last may idle)
  constexpr int BPER = (BRUNS + CNT - 1) / CNT;
  size_t aoff[4];
  int alo[4];
  const uint16_t* asrc[4];
#pragma unroll
  for (int r = 0; r < 4; ++r) {
    const int id = t + CNT * r;
    const int row = id >> 3, hl = (id >> 2) & 1, run = id & 3;
    asrc[r] = hl ? Wl : Wh;
    aoff[r] = static_cast<size_t>(k_lo / KB) * lda + static_cast<size_t>(m0 + row) * KB + run * 8;
    alo[r] = row * 8 + ((hl * 4 + run) ^ sw8(row));
  }
  size_t boff[BPER];
  int blo[BPER];
  const uint16_t* bsrc[BPER];
#pragma unroll
  for (int r = 0; r < BPER; ++r) {
    const int id = t + CNT * r;
    const int row = (id >> 3) < BN ? (id >> 3) : 0, hl = (id >> 2) & 1, run = id & 3;
    bsrc[r] = hl ? Tl : Th;
    boff[r] = static_cast<size_t>(k_lo / KB) * ldb + static_cast<size_t>(n0 + row) * KB + run * 8;
    blo[r] = id < BRUNS ? row * 8 + ((hl * 4 + run) ^ sw8(row)) : -1;
  }
  const int fr = lane & 15, frun = lane >> 4;

  f32x4_t acc[2][NTW];
#pragma unroll
  for (int i = 0; i < 2; ++i)
#pragma unroll
    for (int u = 0; u < NTW; ++u) acc[i][u] = f32x4_t{0.f, 0.f, 0.f, 0.f};

  const long nsteps = k_len / KB;
  u32x4_t ra[4], rb[BPER];
#pragma unroll
  for (int r = 0; r < 4; ++r) ra[r] = *reinterpret_cast<const u32x4_t*>(asrc[r] + aoff[r]);
#pragma unroll
  for (int r = 0; r < BPER; ++r)
    if (blo[r] >= 0) rb[r] = *reinterpret_cast<const u32x4_t*>(bsrc[r] + boff[r]);
#pragma unroll
  for (int r = 0; r < 4; ++r) sA[alo[r]] = ra[r];
#pragma unroll
  for (int r = 0; r < BPER; ++r)
    if (blo[r] >= 0) sB[blo[r]] = rb[r];
  __syncthreads();
  for (long st = 0; st < nsteps; ++st) {
    const int ab = (st & 1) * ARUNS, bb = (st & 1) * BRUNS;
    const bool more = st + 1 < nsteps;
    if (more) {
      const size_t ka = static_cast<size_t>(st + 1) * lda, kb = static_cast<size_t>(st + 1) * ldb;
#pragma unroll
      for (int r = 0; r < 4; ++r) ra[r] = *reinterpret_cast<const u32x4_t*>(asrc[r] + aoff[r] + ka);
#pragma unroll
      for (int r = 0; r < BPER; ++r)
        if (blo[r] >= 0) rb[r] = *reinterpret_cast<const u32x4_t*>(bsrc[r] + boff[r] + kb);
    }
    bf16x8_t a[2][2];
#pragma unroll
    for (int i = 0; i < 2; ++i)
#pragma unroll
      for (int hl = 0; hl < 2; ++hl) {
        const int row = w * 32 + i * 16 + fr;
        a[i][hl] = __builtin_bit_cast(bf16x8_t, sA[ab + row * 8 + ((hl * 4 + frun) ^ sw8(row))]);
      }
#pragma unroll
    for (int u = 0; u < NTW; ++u) {
      const int row = u * 16 + fr, sw = sw8(row);
      const bf16x8_t bh = __builtin_bit_cast(bf16x8_t, sB[bb + row * 8 + ((0 * 4 + frun) ^ sw)]);
      const bf16x8_t bl = __builtin_bit_cast(bf16x8_t, sB[bb + row * 8 + ((1 * 4 + frun) ^ sw)]);
#pragma unroll
      for (int i = 0; i < 2; ++i) acc[i][u] = mfma3(a[i][0], a[i][1], bh, bl, acc[i][u]);
    }
    if (more) {
      const int na = ((st + 1) & 1) * ARUNS, nbb = ((st + 1) & 1) * BRUNS;
#pragma unroll
      for (int r = 0; r < 4; ++r) sA[na + alo[r]] = ra[r];
#pragma unroll
      for (int r = 0; r < BPER; ++r)
        if (blo[r] >= 0) sB[nbb + blo[r]] = rb[r];
    }
    __syncthreads();
  }
  // D[m][n]: lane n + 16*(m/4), element m%4
#pragma unroll
  for (int i = 0; i < 2; ++i)
#pragma unroll
    for (int u = 0; u < NTW; ++u)
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        const long row = m0 + w * 32 + i * 16 + 4 * (lane >> 4) + r;
        float* c = C + row * ncol + n0 + u * 16 + (lane & 15);
        *c = accum ? *c + acc[i][u][r] : acc[i][u][r];
      }
}

// The same product with a square-ish tile: 256 (m) x 64 NSUB (n), eight waves in two
// rows by four columns; wave (wr, wc) owns rows 128 wr .. 128 wr + 127 and columns
// 16 NSUB wc .. + 16 NSUB - 1 (8 x NSUB MFMA tiles), so per k step it reads 16 A and
// 2 NSUB B fragments for 24 NSUB MFMAs (the row strips above read 4 and 2 NTW for 6 NTW).
// LDS holds 16-byte runs [row][8 runs: hl 2 x run 4] as above, double-buffered, but
// with run q of row m at q ^ ((m >> 1) & 7): the sixteen rows of one fragment read still
// hit distinct bank groups, and the swizzle repeats every 16 rows, so the fragments of
// different row tiles lie at constant offsets from one address.  Operands are tiled as
// for contract_bf16x3, and every tile sums its k steps in the same order.
// grid (ncol/(64 NSUB), rows/256, splits), block 512
template <int NSUB>
__global__ __launch_bounds__(512) void contract2_bf16x3(const uint16_t* __restrict__ Wh, const uint16_t* __restrict__ Wl,
                                                        long lda, const uint16_t* __restrict__ Th,
                                                        const uint16_t* __restrict__ Tl, long ldb, long K, int ncol,
                                                        float* __restrict__ C, long kz, long zs, int accum) {
  constexpr int BM = 256, BN = 64 * NSUB, NT = 512;
  constexpr int ARUNS = BM * 8, BRUNS = BN * 8, APER = ARUNS / NT, BPER = BRUNS / NT;
  __shared__ u32x4_t sA[2 * ARUNS];
  __shared__ u32x4_t sB[2 * BRUNS];
  unsigned tx, ty;
  xcd_tile(tx, ty);
  const long n0 = static_cast<long>(tx) * BN, m0 = static_cast<long>(ty) * BM;
  const int t = threadIdx.x, w = t >> 6, lane = t & 63;
  const int wr = w >> 2, wc = w & 3;
  const long k_lo = blockIdx.z * kz;
  const long k_len = (K < k_lo + kz ? K : k_lo + kz) - k_lo;
  C += blockIdx.z * zs;

  // staging: run id t + 512 r is row t/8 + 64 r of the tile, with the thread's own hi/lo
  // array and 8-element run; sw8 of the row does not depend on r
  const int srow = t >> 3, shl = (t >> 2) & 1, srun = t & 3;
  const uint16_t* ap = (shl ? Wl : Wh) + static_cast<size_t>(k_lo / KB) * lda + static_cast<size_t>(m0 + srow) * KB + srun * 8;
  const uint16_t* bp = (shl ? Tl : Th) + static_cast<size_t>(k_lo / KB) * ldb + static_cast<size_t>(n0 + srow) * KB + srun * 8;
  constexpr int astep = 64 * KB, bstep = 64 * KB;  // 64 rows on
  auto sw = [](int m) { return (m >> 1) & 7; };
  const int slo = srow * 8 + ((shl * 4 + srun) ^ sw(srow));  // + 512 r
  const int fr = lane & 15, frun = lane >> 4;

  f32x4_t acc[8][NSUB];
#pragma unroll
  for (int i = 0; i < 8; ++i)
#pragma unroll
    for (int u = 0; u < NSUB; ++u) acc[i][u] = f32x4_t{0.f, 0.f, 0.f, 0.f};

  const long nsteps = k_len / KB;
  u32x4_t ra[APER], rb[BPER];
#pragma unroll
  for (int r = 0; r < APER; ++r) ra[r] = *reinterpret_cast<const u32x4_t*>(ap + r * astep);
#pragma unroll
  for (int r = 0; r < BPER; ++r) rb[r] = *reinterpret_cast<const u32x4_t*>(bp + r * bstep);
#pragma unroll
  for (int r = 0; r < APER; ++r) sA[slo + 512 * r] = ra[r];
#pragma unroll
  for (int r = 0; r < BPER; ++r) sB[slo + 512 * r] = rb[r];
  __syncthreads();
  for (long st = 0; st < nsteps; ++st) {
    const int ab = (st & 1) * ARUNS, bb = (st & 1) * BRUNS;
    const bool more = st + 1 < nsteps;
    if (more) {
      const size_t ka = static_cast<size_t>(st + 1) * lda, kb = static_cast<size_t>(st + 1) * ldb;
#pragma unroll
      for (int r = 0; r < APER; ++r) ra[r] = *reinterpret_cast<const u32x4_t*>(ap + r * astep + ka);
#pragma unroll
      for (int r = 0; r < BPER; ++r) rb[r] = *reinterpret_cast<const u32x4_t*>(bp + r * bstep + kb);
    }
    bf16x8_t bh[NSUB], bl[NSUB];
#pragma unroll
    for (int u = 0; u < NSUB; ++u) {
      const int row = wc * 16 * NSUB + u * 16 + fr;
      bh[u] = __builtin_bit_cast(bf16x8_t, sB[bb + row * 8 + (frun ^ sw(fr))]);
      bl[u] = __builtin_bit_cast(bf16x8_t, sB[bb + row * 8 + ((4 + frun) ^ sw(fr))]);
    }
#pragma unroll
    for (int i = 0; i < 8; ++i) {
      const int row = wr * 128 + i * 16 + fr;
      const bf16x8_t ah = __builtin_bit_cast(bf16x8_t, sA[ab + row * 8 + (frun ^ sw(fr))]);
      const bf16x8_t al = __builtin_bit_cast(bf16x8_t, sA[ab + row * 8 + ((4 + frun) ^ sw(fr))]);
#pragma unroll
      for (int u = 0; u < NSUB; ++u) acc[i][u] = mfma3(ah, al, bh[u], bl[u], acc[i][u]);
    }
    // issue order: the B fragments and the first A pair, then per A row tile its
    // products with the next pair's reads ahead of them
    __builtin_amdgcn_sched_group_barrier(0x100, 2 * NSUB + 2, 0);
#pragma unroll
    for (int i = 0; i < 7; ++i) {
      __builtin_amdgcn_sched_group_barrier(0x008, 3 * NSUB, 0);
      __builtin_amdgcn_sched_group_barrier(0x100, 2, 0);
    }
    __builtin_amdgcn_sched_group_barrier(0x008, 3 * NSUB, 0);
    if (more) {
      const int na = ((st + 1) & 1) * ARUNS, nbb = ((st + 1) & 1) * BRUNS;
#pragma unroll
      for (int r = 0; r < APER; ++r) sA[na + slo + 512 * r] = ra[r];
#pragma unroll
      for (int r = 0; r < BPER; ++r) sB[nbb + slo + 512 * r] = rb[r];
    }
    __syncthreads();
  }
  // D[m][n]: lane n + 16*(m/4), element m%4
#pragma unroll
  for (int i = 0; i < 8; ++i)
#pragma unroll
    for (int u = 0; u < NSUB; ++u)
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        const long row = m0 + wr * 128 + i * 16 + 4 * (lane >> 4) + r;
        float* c = C + row * ncol + n0 + wc * 16 * NSUB + u * 16 + (lane & 15);
        *c = accum ? *c + acc[i][u][r] : acc[i][u][r];
      }
}

// ---------------------------------------------------------------- slot order
// Tn = T with the slots of every block pair in natural order: element (n, 256 q + 16 x + y)
// of Tn is element (n, 256 q + split_slot(x, y)) of T (16-bit words; both tiled in 32
// slots, ncol = gridDim.y rows).  grid (K/256, ncol), block 256
__global__ __launch_bounds__(256) void natural_slots_u16(const uint16_t* __restrict__ T, uint16_t* __restrict__ Tn) {
  const size_t n = blockIdx.y, ts = static_cast<size_t>(gridDim.y) * KB;
  const int nu = threadIdx.x;
  const size_t kd = static_cast<size_t>(blockIdx.x) * 256 + nu;
  const size_t ks = static_cast<size_t>(blockIdx.x) * 256 + split_slot(nu >> 4, nu & 15);
  Tn[kd / KB * ts + n * KB + kd % KB] = T[ks / KB * ts + n * KB + ks % KB];
}

// ---------------------------------------------------------------- transpose
// dst (r', k') = src (k', r') for the 32 x 32 tiles of two tiled operands: src element
// (r, k) at (k / 32) * sts + r * 32 + k % 32, dst element (r', k') at (k' / 32) * dts +
// r' * 32 + k' % 32 (16-bit words).  One workgroup moves one contiguous 2 KB tile to
// another.  grid (dst rows / 32, src rows / 32), block 256
__global__ __launch_bounds__(256) void transpose_tiles_u16(const uint16_t* __restrict__ src, long sts,
                                                           uint16_t* __restrict__ dst, long dts) {
  __shared__ uint16_t tile[32][34];
  const size_t kt = blockIdx.x, rt = blockIdx.y;  // src k tile (= dst row tile), src row tile
  const int t = threadIdx.x, r = t >> 3, c = (t & 7) * 4;
  const uint16_t* s = src + kt * sts + rt * (32 * KB);
  uint16_t* d = dst + rt * dts + kt * (32 * KB);
  const uint2 x = *reinterpret_cast<const uint2*>(s + r * KB + c);
  tile[r][c] = static_cast<uint16_t>(x.x);
  tile[r][c + 1] = static_cast<uint16_t>(x.x >> 16);
  tile[r][c + 2] = static_cast<uint16_t>(x.y);
  tile[r][c + 3] = static_cast<uint16_t>(x.y >> 16);
  __syncthreads();
  // dst row r (= src k c0 + r), columns c .. c + 3 (= src rows)
  uint2 y;
  y.x = static_cast<uint32_t>(tile[c][r]) | (static_cast<uint32_t>(tile[c + 1][r]) << 16);
  y.y = static_cast<uint32_t>(tile[c + 2][r]) | (static_cast<uint32_t>(tile[c + 3][r]) << 16);
  *reinterpret_cast<uint2*>(d + r * KB + c) = y;
}

// ---------------------------------------------------------------- split sums
// dst[i] = (accum ? dst[i] : 0) + (sum over z < nz of P[z * zs + i], added in z order),
// for i < n (n and zs multiples of 4, arrays 16-byte aligned).  Four partials are read
// together (clamped to a valid split, the extra ones not added).
// grid ceil(n / 1024), block 256
__global__ __launch_bounds__(256) void sum_splits_f32(const float* __restrict__ P, long zs, int nz, long n,
                                                      float* __restrict__ dst, int accum) {
  const long i = (static_cast<long>(blockIdx.x) * 256 + threadIdx.x) * 4;
  if (i >= n) return;
  f32x4_t acc = f32x4_t{0.f, 0.f, 0.f, 0.f};
  for (int z = 0; z < nz; z += 4) {
    f32x4_t x[4];
#pragma unroll
    for (int k = 0; k < 4; ++k) {
      const long zk = z + k < nz ? z + k : nz - 1;
      x[k] = *reinterpret_cast<const f32x4_t*>(P + zk * zs + i);
    }
#pragma unroll
    for (int k = 0; k < 4; ++k)
      if (z + k < nz) acc = z + k == 0 ? x[k] : acc + x[k];
  }
  f32x4_t* d = reinterpret_cast<f32x4_t*>(dst + i);
  *d = accum ? *d + acc : acc;
}

// ---------------------------------------------------------------- host
// Workgroups of the contraction kernel for (wide, ntw) resident at once on the device.
static long contract_slots(int wide, int ntw) {
  const void* f;
  if (wide) {
    f = ntw == 8    ? reinterpret_cast<const void*>(&contract2_bf16x3<2>)
        : ntw == 12 ? reinterpret_cast<const void*>(&contract2_bf16x3<3>)
                    : reinterpret_cast<const void*>(&contract2_bf16x3<4>);
    return resident_wgs(f, 512, 1);
  }
  switch (ntw) {
    case 1: f = reinterpret_cast<const void*>(&contract_bf16x3<1>); break;
    case 2: f = reinterpret_cast<const void*>(&contract_bf16x3<2>); break;
    case 3: f = reinterpret_cast<const void*>(&contract_bf16x3<3>); break;
    case 4: f = reinterpret_cast<const void*>(&contract_bf16x3<4>); break;
    case 5: f = reinterpret_cast<const void*>(&contract_bf16x3<5>); break;
    case 6: f = reinterpret_cast<const void*>(&contract_bf16x3<6>); break;
    case 7: f = reinterpret_cast<const void*>(&contract_bf16x3<7>); break;
    case 8: f = reinterpret_cast<const void*>(&contract_bf16x3<8>); break;
    default: f = reinterpret_cast<const void*>(&contract_bf16x3<9>); break;
  }
  return resident_wgs(f, CNT, 1);
}

// Splits of the contraction's k range for a launch of `rows` rows and 16*ntw-wide
// column tiles (wide: the 256 x 64 NSUB kernel): at least one full round of resident
// workgroups, and enough that one split's slice of the packed amplitudes (hi and lo
// words, ncol rows of K/z) stays within RI_PPL_TAU_CHUNK_MB (default TAU_CHUNK_MB), for
// the reason given with the FP64 path's splits; then balanced so that the last round of
// workgroups is not a few stragglers.  At least 32 steps per split.  kz: summed indices
// per split.
static int contract_splits(int wide, int ntw, int ncol, long rows, long K, long& kz) {
  const long nwg = (ncol / (16 * ntw)) * (rows / CBM);
  const long slots = contract_slots(wide, ntw);
  long z = (slots + nwg - 1) / nwg;
  const double chunk = static_cast<double>(env_long("RI_PPL_TAU_CHUNK_MB", TAU_CHUNK_MB)) * 1048576.0;
  z = std::max(z, static_cast<long>(std::ceil(static_cast<double>(K) * ncol * 4.0 / chunk)));
  const long zmax = std::max(1L, K / (32 * KB));
  z = std::max(1L, std::min(z, zmax));
  z = balance_splits(nwg, slots, K, KB, z, zmax);
  kz = (K + z - 1) / z;
  kz = (kz + KB - 1) / KB * KB;
  return static_cast<int>((K + kz - 1) / kz);
}

// Splits of the exchange-symmetric form's second product (k = the slab's M slots, rows2
// rows): enough to fill the chip once, at least 8 steps per split, balanced as above,
// and no more than `avail` elements of partial sums (rows2 * ncol per split) hold.
static int second_splits(int wide, int ntw, int ncol, long rows2, long M, size_t avail, long& kz) {
  const long nwg = (ncol / (16 * ntw)) * (rows2 / CBM);
  const long slots = contract_slots(wide, ntw);
  const long zmax = std::max(1L, std::min(M / (8 * KB), static_cast<long>(avail / (static_cast<size_t>(rows2) * ncol))));
  long z = std::max(1L, std::min((slots + nwg - 1) / nwg, zmax));
  z = balance_splits(nwg, slots, M, KB, z, zmax);
  kz = (M + z - 1) / z;
  kz = (kz + KB - 1) / KB * KB;
  return static_cast<int>((M + kz - 1) / kz);
}

struct MPlan {
  int o, v, naux, nb, vp, Qp;
  long nbp, K;
  int po, pm, NP, NM, ntw_p, ntw_m;
  int wide_p, wide_m;  // 1: contract2_bf16x3 with NSUB = ntw / 4 for that side
  long slab_bp, slab_M;
  size_t n_B, n_Tp, n_Tm, n_W, n_S, n_A;  // element counts
  long zrows_p, zrows_m;                   // largest splits x rows of one contraction launch
  size_t bytes;
};

// Largest splits x rows over the slab sizes of plan p (the full slab and the last).
static long max_split_rows(const MPlan& p, int wide, int ncol, int ntw) {
  if (ncol == 0) return 0;
  long kz;
  const long last = p.nbp - (p.nbp - 1) / p.slab_bp * p.slab_bp;
  long best = 0;
  for (long rows : {p.slab_M, last * 256})
    best = std::max(best, contract_splits(wide, ntw, ncol, rows, p.K, kz) * rows);
  return best;
}

// Element counts and total bytes of plan p for its slab width p.slab_bp.
static void size_mplan(MPlan& p) {
  p.slab_M = p.slab_bp * 256;
  p.n_B = static_cast<size_t>(p.vp) * p.vp * p.Qp;
  p.n_Tp = static_cast<size_t>(p.NP) * p.K;
  p.n_Tm = static_cast<size_t>(p.NM) * p.K;
  p.n_W = static_cast<size_t>(p.slab_M) * p.K;
  p.zrows_p = max_split_rows(p, p.wide_p, p.NP, p.ntw_p);
  p.zrows_m = max_split_rows(p, p.wide_m, p.NM, p.ntw_m);
  p.n_S = static_cast<size_t>(p.zrows_p) * p.NP;
  p.n_A = static_cast<size_t>(p.zrows_m) * p.NM;
  size_t b = 0;
  // 16-bit: Bh, Bl, Tph, Tpl, Tmh, Tml, Wph, Wpl, Wmh, Wml; 32-bit: S, A
  for (size_t n : {p.n_B, p.n_B, p.n_Tp, p.n_Tp, p.n_Tm, p.n_Tm, p.n_W, p.n_W, p.pm > 0 ? p.n_W : 0,
                   p.pm > 0 ? p.n_W : 0})
    b = round_up(b, 256) + n * 2;
  for (size_t n : {p.n_S, p.n_A}) b = round_up(b, 256) + n * 4;
  p.bytes = round_up(b, 256);
}

// fit_bytes > 0: the widest slab whose whole workspace fits in fit_bytes (false if not
// even a one-block-pair slab fits), instead of the W budget RI_PPL_W_BYTES.
static bool make_mplan(int o, int v, int naux, MPlan& p, size_t fit_bytes = 0) {
  if (o <= 0 || v <= 0 || naux <= 0 || o > 4096 || v > 65536 || naux > (1 << 24)) return false;
  p.o = o;
  p.v = v;
  p.naux = naux;
  p.nb = (v + TB - 1) / TB;
  p.vp = p.nb * TB;
  p.Qp = static_cast<int>(round_up(naux, QC));
  // the build's buffer loads reach eight factor rows of vp * Qp bf16 words past their
  // base with 32-bit byte offsets
  if (static_cast<double>(p.vp) * p.Qp * 2 * 8 >= 2147483648.0) return false;
  p.nbp = static_cast<long>(p.nb) * (p.nb + 1) / 2;
  p.K = p.nbp * 256;
  p.po = o * (o + 1) / 2;
  p.pm = o * (o - 1) / 2;
  // per side: the 256 x 64 NSUB tiles (NSUB 4, 3 or 2, the fewest padded columns, ties
  // to the wider) unless they pad to more columns than the row strips
  auto pick = [](int ncols, int& ntw, int& padded, int& wide) {
    int sntw, spad;
    pick_ntw(ncols, 9, CBM, sntw, spad);
    int tpad = 1 << 30, tntw = 16;
    for (int ns : {4, 3, 2}) {
      const int w = 64 * ns, pad = std::max(1, (ncols + w - 1) / w) * w;
      if (pad < tpad) {
        tpad = pad;
        tntw = 4 * ns;
      }
    }
    wide = tpad <= spad ? 1 : 0;
    ntw = wide ? tntw : sntw;
    padded = wide ? tpad : spad;
  };
  pick(p.po, p.ntw_p, p.NP, p.wide_p);
  pick(p.pm, p.ntw_m, p.NM, p.wide_m);
  if (p.pm == 0) p.NM = 0;
  const int nw = p.pm > 0 ? 2 : 1;
  const long budget = env_long("RI_PPL_W_BYTES", 16L << 30);
  long bp = budget / (static_cast<long>(nw) * p.K * 256 * 4);
  bp = std::max(1L, std::min(bp, std::min(p.nbp, 65535L)));
  if (fit_bytes > 0) bp = std::min(p.nbp, 65535L);
  const long cap = env_long("RI_PPL_SLAB_PAIRS", bp);
  p.slab_bp = std::min(cap, bp);
  size_mplan(p);
  if (fit_bytes > 0 && p.bytes > fit_bytes) {  // bytes grow with the slab width: bisect
    long lo = 1, hi = p.slab_bp - 1;
    p.slab_bp = 1;
    size_mplan(p);
    if (p.bytes > fit_bytes) return false;
    while (lo < hi) {
      const long mid = (lo + hi + 1) / 2;
      p.slab_bp = mid;
      size_mplan(p);
      if (p.bytes <= fit_bytes) lo = mid; else hi = mid - 1;
    }
    p.slab_bp = lo;
    size_mplan(p);
  }
  return true;
}

// The k range (extent K) is split `splits` ways (kz each) into partial outputs rows*ncol
// apart.  lda, ldb: elements from one tile of KB k of the operand to the next.
struct CArgs {
  const uint16_t *Wh, *Wl;
  long lda;
  const uint16_t *Th, *Tl;
  long ldb, K, rows;
  int ncol;
  float* C;
  int splits;
  long kz;
  int accum;
};
template <int NTW>
static void launch_c(const CArgs& a, hipStream_t s) {
  contract_bf16x3<NTW><<<dim3(a.ncol / (16 * NTW), a.rows / CBM, a.splits), CNT, 0, s>>>(
      a.Wh, a.Wl, a.lda, a.Th, a.Tl, a.ldb, a.K, a.ncol, a.C, a.kz, a.rows * a.ncol, a.accum);
}

template <int NSUB>
static void launch_c2(const CArgs& a, hipStream_t s) {
  contract2_bf16x3<NSUB><<<dim3(a.ncol / (64 * NSUB), a.rows / CBM, a.splits), 512, 0, s>>>(
      a.Wh, a.Wl, a.lda, a.Th, a.Tl, a.ldb, a.K, a.ncol, a.C, a.kz, a.rows * a.ncol, a.accum);
}

static void launch_contract(int wide, int ntw, const CArgs& a, hipStream_t s) {
  if (wide) {
    switch (ntw) {
      case 8: launch_c2<2>(a, s); break;
      case 12: launch_c2<3>(a, s); break;
      default: launch_c2<4>(a, s); break;
    }
    return;
  }
  switch (ntw) {
    case 1: launch_c<1>(a, s); break;
    case 2: launch_c<2>(a, s); break;
    case 3: launch_c<3>(a, s); break;
    case 4: launch_c<4>(a, s); break;
    case 5: launch_c<5>(a, s); break;
    case 6: launch_c<6>(a, s); break;
    case 7: launch_c<7>(a, s); break;
    case 8: launch_c<8>(a, s); break;
    default: launch_c<9>(a, s); break;
  }
}

// Off-diagonal build of the slab's ab block pairs [slab0, slab0 + npairs) against cd
// block pairs pcd0 .. nbp-1, in the grouped workgroup order: one ab block pair by a
// 4 x 4 tile of cd block pairs, i.e. 32 workgroups, one per CU of an XCD (at o=48
// v=768 naux=2304 2% faster than 2 x 2 or 8 x 8 tiles and than runs of 32 consecutive
// cd halves).
constexpr int GROUP_AB = 1, GROUP_T = 4;
static void launch_build(const uint16_t* Bh, const uint16_t* Bl, const MPlan& p, long slab0, long npairs, long pcd0,
                         uint16_t* Wph, uint16_t* Wpl, uint16_t* Wmh, uint16_t* Wml, hipStream_t s) {
  const long nb = p.vp / TB, nT = (nb + GROUP_T - 1) / GROUP_T;
  int C0, D0;
  tri_decode(pcd0, C0, D0);
  const long k0 = D0 / GROUP_T, ntile = nT * (nT + 1) / 2 - k0 * (k0 + 1) / 2;
  const long ngroups = ntile * ((npairs + GROUP_AB - 1) / GROUP_AB);
  const long nwg = (ngroups + 7) / 8 * 8 * GROUP_AB * 2L * GROUP_T * GROUP_T;
  build_w_bf16x3<<<dim3(static_cast<unsigned>(nwg)), 512, 0, s>>>(Bh, Bl, p.Qp, p.vp, slab0, npairs * 256 * KB,
                                                                   p.pm > 0 ? 1 : 0,
                                                                   pcd0, npairs, GROUP_AB, GROUP_T, Wph, Wpl, Wmh,
                                                                   Wml);
}

size_t bf16x3_workspace_bytes(int o, int v, int naux) {
  MPlan p;
  return make_mplan(o, v, naux, p) ? p.bytes : 0;
}

size_t bf16x3_workspace_bytes_min(int o, int v, int naux) {
  MPlan p;
  if (!make_mplan(o, v, naux, p)) return 0;
  p.slab_bp = 1;
  size_mplan(p);
  return p.bytes;
}

int bf16x3_run(const double* B, long qs, long rs, const double* tau, int o, int v, int naux, double* R, void* ws,
               size_t ws_bytes, int shard, int nshards, hipStream_t s, bool fit) {
  MPlan p;
  if (!make_mplan(o, v, naux, p, fit ? ws_bytes : 0)) {
    if (fit && make_mplan(o, v, naux, p)) {
      set_error("ladder: no slab plan for o=%d v=%d naux=%d fits %zu bytes of workspace", o, v, naux, ws_bytes);
      return RI_E_NOMEM;
    }
    set_error("ladder: invalid sizes o=%d v=%d naux=%d", o, v, naux);
    return RI_E_ARG;
  }
  void* buf = ws;
  bool own = false;
  if (!buf) {
    RI_TRY(dev_alloc(&buf, p.bytes, s));
    own = true;
  } else if (ws_bytes < p.bytes) {
    set_error("ladder: workspace of %zu bytes is smaller than the %zu required", ws_bytes, p.bytes);
    return RI_E_NOMEM;
  }
  Carve cv(buf, p.bytes);
  uint16_t* Bh = cv.take<uint16_t>(p.n_B);
  uint16_t* Bl = cv.take<uint16_t>(p.n_B);
  uint16_t* Tph = cv.take<uint16_t>(p.n_Tp);
  uint16_t* Tpl = cv.take<uint16_t>(p.n_Tp);
  uint16_t* Tmh = cv.take<uint16_t>(p.n_Tm);
  uint16_t* Tml = cv.take<uint16_t>(p.n_Tm);
  uint16_t* Wph = cv.take<uint16_t>(p.n_W);
  uint16_t* Wpl = cv.take<uint16_t>(p.n_W);
  uint16_t* Wmh = cv.take<uint16_t>(p.pm > 0 ? p.n_W : 0);
  uint16_t* Wml = cv.take<uint16_t>(p.pm > 0 ? p.n_W : 0);
  float* S = cv.take<float>(p.n_S);
  float* A = cv.take<float>(p.n_A);

  int rc = RI_OK;
  const double vv = static_cast<double>(v) * v, oo = static_cast<double>(o) * o;
  const double pv = v * (v + 1.0) / 2, pvm = v * (v - 1.0) / 2;
  do {
    {
      ProfScope ps(s, "split_b_bf16", 0.0, 8.0 * vv * naux + 4.0 * vv * naux);
      split_b_kernel<<<dim3(p.Qp / 32, p.vp / 32 + (p.vp % 32 ? 1 : 0), p.vp), 256, 0, s>>>(B, qs, rs, v, naux, p.vp,
                                                                                           p.Qp, Bh, Bl);
      if ((rc = check_launch("split_b_kernel"))) break;
    }
    {
      ProfScope ps(s, "pack_tau_bf16", 0.0, 8.0 * oo * vv + 4.0 * (pv * p.po + pvm * p.pm));
      pack_tau_bf16_kernel<<<dim3(p.nbp, p.NP), 256, 0, s>>>(tau, o, v, +1, Tph, Tpl);
      if ((rc = check_launch("pack_tau_bf16(+)"))) break;
      if (p.pm > 0) {
        pack_tau_bf16_kernel<<<dim3(p.nbp, p.NM), 256, 0, s>>>(tau, o, v, -1, Tmh, Tml);
        if ((rc = check_launch("pack_tau_bf16(-)"))) break;
      }
    }
    for (long slab0 = 0; slab0 < p.nbp && rc == RI_OK; slab0 += p.slab_bp) {
      if ((slab0 / p.slab_bp) % nshards != shard) continue;  // another shard's slab
      const long npairs = std::min(p.slab_bp, p.nbp - slab0);
      const long M = npairs * 256;
      double le, lt, ld;
      count_pairs(v, slab0, npairs, le, lt, ld);
      int dy0, ndiag;
      diag_pairs(slab0, npairs, dy0, ndiag);
      long kzp = 0, kzm = 0;
      const int zp = contract_splits(p.wide_p, p.ntw_p, p.NP, M, p.K, kzp);
      const int zm = p.pm > 0 ? contract_splits(p.wide_m, p.ntw_m, p.NM, M, p.K, kzm) : 1;
      {  // off-diagonal and diagonal ab block pairs in two launches
        ProfScope ps(s, "build_w_bf16x3", 2.0 * naux * vv * (le - ld));
        launch_build(Bh, Bl, p, slab0, npairs, 0, Wph, Wpl, Wmh, Wml, s);
        if ((rc = check_launch("build_w_bf16x3"))) break;
      }
      if (ndiag > 0) {
        ProfScope ps(s, "build_w_bf16x3_diag", 2.0 * naux * vv * ld);
        build_w_bf16x3_diag<<<dim3(p.nbp * 2, ndiag), 512, 0, s>>>(Bh, Bl, p.Qp, p.vp, slab0, M * KB,
                                                                   p.pm > 0 ? 1 : 0, dy0, 0, Wph, Wpl, Wmh, Wml);
        if ((rc = check_launch("build_w_bf16x3_diag"))) break;
      }
      {
        ProfScope ps(s, "contract_bf16x3", 2.0 * (le * pv * p.po + lt * pvm * p.pm));
        launch_contract(p.wide_p, p.ntw_p, CArgs{Wph, Wpl, M * KB, Tph, Tpl, p.NP * KB, p.K, M, p.NP, S, zp, kzp, 0}, s);
        if ((rc = check_launch("contract_bf16x3(+)"))) break;
        if (p.pm > 0) {
          launch_contract(p.wide_m, p.ntw_m, CArgs{Wmh, Wml, M * KB, Tmh, Tml, p.NM * KB, p.K, M, p.NM, A, zm, kzm, 0}, s);
          if ((rc = check_launch("contract_bf16x3(-)"))) break;
        }
      }
      {
        ProfScope ps(s, "unpack_f32", 0.0, 16.0 * oo * (le + lt));
        launch_unpack_f32(S, A, p.NP, p.NM, o, v, slab0, npairs, R, zp, M * p.NP, zm, M * p.NM, s);
        if ((rc = check_launch("unpack_f32"))) break;
      }
    }
  } while (false);
  if (own) dev_free(buf, s);
  return rc;
}

// ---------------------------------------------------------------- exchange symmetry
// The exchange-symmetric ladder (factors symmetric in their virtual indices) in split
// bf16: as the FP64 form, slab [P0, P1) builds the cd block pairs >= P0 only and uses
// each built element twice.  W here is W[ab slot][cd slot] (tiled in 32 cd slots), so
// for the second product
//   S2[cd][n] += sum_{ab in slab} W[ab][cd] T[n][ab]        (rows cd >= P1)
// the block W[:, P1*256:] is first transposed (transpose_tiles_u16, 16-bit words) into
// W2[cd][ab], after which the product is the contraction kernel with the slab's slice of
// T, accumulating into S2 in slab order.  The ab index of W is in natural slot order and
// its cd index in the split order (split_slot), so the second product sums against a
// natural-order copy of T and leaves S2's rows in the split order, which the final
// unpack reads as such.  S2 and A2 are FP32 and unpacked once at the end.
// slab_bp: the slab width (block pairs), the same for every precision of this form.
int bf16x3_run_sym(const double* B, const double* tau, int o, int v, int naux, double* R, long slab_bp,
                   hipStream_t s) {
  MPlan p;
  if (!make_mplan(o, v, naux, p)) {
    set_error("ri_ppl_sym: invalid sizes o=%d v=%d naux=%d", o, v, naux);
    return RI_E_ARG;
  }
  p.slab_bp = std::max(1L, std::min(slab_bp, p.nbp));
  size_mplan(p);
  const size_t n_S2 = static_cast<size_t>(p.K) * p.NP, n_A2 = static_cast<size_t>(p.K) * p.NM;
  const size_t n_W2 = p.n_W;  // (K - P1*256) x M <= K x slab_M per array
  const int nw = p.pm > 0 ? 4 : 2;
  const size_t bytes = p.bytes + round_up(n_S2 * 4, 256) + round_up(n_A2 * 4, 256) + nw * round_up(n_W2 * 2, 256) +
                       2 * round_up(p.n_Tp * 2, 256) + 2 * round_up(p.n_Tm * 2, 256);
  void* buf = nullptr;
  RI_TRY(dev_alloc(&buf, bytes, s));
  Carve cv(buf, bytes);
  uint16_t* Bh = cv.take<uint16_t>(p.n_B);
  uint16_t* Bl = cv.take<uint16_t>(p.n_B);
  uint16_t* Tph = cv.take<uint16_t>(p.n_Tp);
  uint16_t* Tpl = cv.take<uint16_t>(p.n_Tp);
  uint16_t* Tmh = cv.take<uint16_t>(p.n_Tm);
  uint16_t* Tml = cv.take<uint16_t>(p.n_Tm);
  uint16_t* Wph = cv.take<uint16_t>(p.n_W);
  uint16_t* Wpl = cv.take<uint16_t>(p.n_W);
  uint16_t* Wmh = cv.take<uint16_t>(p.pm > 0 ? p.n_W : 0);
  uint16_t* Wml = cv.take<uint16_t>(p.pm > 0 ? p.n_W : 0);
  float* S = cv.take<float>(p.n_S);
  float* A = cv.take<float>(p.n_A);
  float* S2 = cv.take<float>(n_S2);
  float* A2 = cv.take<float>(n_A2);
  uint16_t* W2[4];
  for (int k = 0; k < nw; ++k) W2[k] = cv.take<uint16_t>(n_W2);
  uint16_t* Tnph = cv.take<uint16_t>(p.n_Tp);  // natural slot order
  uint16_t* Tnpl = cv.take<uint16_t>(p.n_Tp);
  uint16_t* Tnmh = cv.take<uint16_t>(p.n_Tm);
  uint16_t* Tnml = cv.take<uint16_t>(p.n_Tm);

  int rc = RI_OK;
  const double oo = static_cast<double>(o) * o;
  const double vv = static_cast<double>(v) * v;
  const long qs = static_cast<long>(v) * v, rs = v;
  do {
    {
      ProfScope ps(s, "split_b_bf16", 0.0, 8.0 * vv * naux + 4.0 * vv * naux);
      split_b_kernel<<<dim3(p.Qp / 32, p.vp / 32 + (p.vp % 32 ? 1 : 0), p.vp), 256, 0, s>>>(B, qs, rs, v, naux, p.vp,
                                                                                           p.Qp, Bh, Bl);
      if ((rc = check_launch("split_b_kernel"))) break;
    }
    {
      ProfScope ps(s, "pack_tau_bf16", 0.0, 0.0);
      pack_tau_bf16_kernel<<<dim3(p.nbp, p.NP), 256, 0, s>>>(tau, o, v, +1, Tph, Tpl);
      if ((rc = check_launch("pack_tau_bf16(+)"))) break;
      if (p.pm > 0) {
        pack_tau_bf16_kernel<<<dim3(p.nbp, p.NM), 256, 0, s>>>(tau, o, v, -1, Tmh, Tml);
        if ((rc = check_launch("pack_tau_bf16(-)"))) break;
      }
      const dim3 gp(static_cast<unsigned>(p.nbp), p.NP), gm(static_cast<unsigned>(p.nbp), p.NM);
      natural_slots_u16<<<gp, 256, 0, s>>>(Tph, Tnph);
      natural_slots_u16<<<gp, 256, 0, s>>>(Tpl, Tnpl);
      if (p.pm > 0) {
        natural_slots_u16<<<gm, 256, 0, s>>>(Tmh, Tnmh);
        natural_slots_u16<<<gm, 256, 0, s>>>(Tml, Tnml);
      }
      if ((rc = check_launch("natural_slots_u16"))) break;
    }
    long first_p1 = -1;
    for (long slab0 = 0; slab0 < p.nbp && rc == RI_OK; slab0 += p.slab_bp) {
      const long npairs = std::min(p.slab_bp, p.nbp - slab0), p1 = slab0 + npairs;
      const long M = npairs * 256, K1 = p.K - slab0 * 256;
      double le, lt, ld, ce, ct, cd;
      count_pairs(v, slab0, npairs, le, lt, ld);
      count_pairs(v, slab0, p.nbp - slab0, ce, ct, cd);
      int dy0, ndiag;
      diag_pairs(slab0, npairs, dy0, ndiag);
      const double per_ab = 2.0 * naux * (2.0 * ct + (ce - ct));
      {
        ProfScope ps(s, "build_w_bf16x3", per_ab * (le - ld));
        launch_build(Bh, Bl, p, slab0, npairs, slab0, Wph, Wpl, Wmh, Wml, s);
        if ((rc = check_launch("build_w_bf16x3"))) break;
      }
      if (ndiag > 0) {
        ProfScope ps(s, "build_w_bf16x3_diag", per_ab * ld);
        build_w_bf16x3_diag<<<dim3((p.nbp - slab0) * 2, ndiag), 512, 0, s>>>(Bh, Bl, p.Qp, p.vp, slab0, M * KB,
                                                                             p.pm > 0 ? 1 : 0, dy0, slab0, Wph, Wpl,
                                                                             Wmh, Wml);
        if ((rc = check_launch("build_w_bf16x3_diag"))) break;
      }
      long kzp = 0, kzm = 0;
      const int zp = contract_splits(p.wide_p, p.ntw_p, p.NP, M, K1, kzp);
      const int zm = p.pm > 0 ? contract_splits(p.wide_m, p.ntw_m, p.NM, M, K1, kzm) : 1;
      const size_t c0 = static_cast<size_t>(slab0) * 256;  // first cd slot built for the slab
      {
        ProfScope ps(s, "contract_bf16x3", 2.0 * (le * ce * p.po + lt * ct * p.pm));
        launch_contract(p.wide_p, p.ntw_p, CArgs{Wph + c0 * M, Wpl + c0 * M, M * KB, Tph + c0 * p.NP, Tpl + c0 * p.NP, p.NP * KB, K1, M, p.NP, S, zp, kzp, 0}, s);
        if ((rc = check_launch("contract_bf16x3(+)"))) break;
        if (p.pm > 0) {
          launch_contract(p.wide_m, p.ntw_m, CArgs{Wmh + c0 * M, Wml + c0 * M, M * KB, Tmh + c0 * p.NM, Tml + c0 * p.NM, p.NM * KB, K1, M, p.NM, A, zm, kzm, 0},
                          s);
          if ((rc = check_launch("contract_bf16x3(-)"))) break;
        }
      }
      {
        ProfScope ps(s, "unpack_f32", 0.0, 16.0 * oo * (le + lt));
        launch_unpack_f32(S, A, p.NP, p.NM, o, v, slab0, npairs, R, zp, M * p.NP, zm, M * p.NM, s);
        if ((rc = check_launch("unpack_f32"))) break;
      }
      if (p1 < p.nbp) {  // second product over the rows cd >= P1
        const long rows2 = (p.nbp - p1) * 256;
        const size_t c1 = static_cast<size_t>(p1) * 256;
        const int accum = first_p1 < 0 ? 0 : 1;
        if (first_p1 < 0) first_p1 = p1;
        {
          ProfScope ps(s, "transpose_w_bf16", 0.0, 4.0 * nw * static_cast<double>(M) * rows2);
          uint16_t* Ws[4] = {Wph, Wpl, Wmh, Wml};
          for (int k = 0; k < nw; ++k)
            transpose_tiles_u16<<<dim3(static_cast<unsigned>(rows2 / 32), static_cast<unsigned>(M / 32)), 256, 0, s>>>(
                Ws[k] + c1 * M, M * KB, W2[k], rows2 * KB);
          if ((rc = check_launch("transpose_tiles_u16"))) break;
        }
        double le2, lt2, ld2;
        count_pairs(v, p1, p.nbp - p1, le2, lt2, ld2);
        ProfScope ps(s, "second_product_bf16x3", 2.0 * (le2 * le * p.po + lt2 * lt * p.pm));
        // split over the slab's slots into the partial buffers S and A (free once the
        // first product is unpacked), then added into S2 and A2 in split order; one
        // split accumulates into S2 and A2 directly
        const int nside = p.pm > 0 ? 2 : 1;
        for (int side = 0; side < nside && rc == RI_OK; ++side) {
          const bool plus = side == 0;
          const int wide = plus ? p.wide_p : p.wide_m, ntw = plus ? p.ntw_p : p.ntw_m, ncol = plus ? p.NP : p.NM;
          float* part = plus ? S : A;
          float* dst = (plus ? S2 : A2) + c1 * ncol;
          long kz2;
          const int z2 = second_splits(wide, ntw, ncol, rows2, M, plus ? p.n_S : p.n_A, kz2);
          const uint16_t* Th = plus ? Tnph : Tnmh;
          const uint16_t* Tl = plus ? Tnpl : Tnml;
          const CArgs ca{W2[plus ? 0 : 2], W2[plus ? 1 : 3], rows2 * KB, Th + c0 * ncol, Tl + c0 * ncol, ncol * KB, M,
                         rows2, ncol, z2 > 1 ? part : dst, z2, kz2, z2 > 1 ? 0 : accum};
          launch_contract(wide, ntw, ca, s);
          if ((rc = check_launch(plus ? "second product (+)" : "second product (-)"))) break;
          if (z2 > 1) {
            const long n = rows2 * ncol;
            sum_splits_f32<<<dim3(static_cast<unsigned>((n + 1023) / 1024)), 256, 0, s>>>(part, n, z2, n, dst, accum);
            rc = check_launch("sum_splits_f32");
          }
        }
        if (rc != RI_OK) break;
      }
    }
    if (rc == RI_OK && first_p1 >= 0) {
      const long n2 = p.nbp - first_p1;
      double le, lt, ld;
      count_pairs(v, first_p1, n2, le, lt, ld);
      ProfScope ps(s, "unpack_f32", 0.0, 16.0 * oo * (le + lt));
      launch_unpack_f32(S2 + static_cast<size_t>(first_p1) * 256 * p.NP,
                        A2 + static_cast<size_t>(first_p1) * 256 * p.NM, p.NP, p.NM, o, v, first_p1, n2, R, 1, 0, 1, 0,
                        s, 1);
      rc = check_launch("unpack_f32");
    }
  } while (false);
  dev_free(buf, s);
  return rc;
}

}  // namespace ppl
}  // namespace ri
