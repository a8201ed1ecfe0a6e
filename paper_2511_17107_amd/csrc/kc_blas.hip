// Tall-skinny block kernels of the LOBPCG iteration on gfx950: complex Gram products on FP64
// MFMA, in-place block updates on FP64 MFMA, the fused residual/preconditioner pass and the
// seeded initial block.
//
// Block storage (per k-point b of a batch): column c of a block lives at base + (b*kstride + c)*n,
// n = 3N^3 complex128 entries per column (one k-space vector, [3][N^3]).
//
// v_mfma_f64_16x16x4f64 computes D(16x16) += A(16x4) B(4x16): lane l supplies A[l%16][l/16]
// and B[l/16][l%16] and holds D[l/16 + 4r][l%16], r = 0..3, afterwards.
#include <algorithm>

#include "kc_blas.h"

namespace kc {

typedef double d4 __attribute__((ext_vector_type(4)));

__device__ __forceinline__ d4 mfma(double a, double b, d4 c) {
  return __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, c, 0, 0, 0);
}

// ------------------------------------------------------------------------------------
// Gram matrices of the Rayleigh-Ritz step: GA_b = S_b^H AS_b and GB_b = S_b^H S_b (nc x nc,
// Hermitian: only the 16x16 tiles on and above the diagonal are formed).  Complex products on
// real MFMA: with a = ar + i ai, b = br + i bi,
//   Re(conj(a) b) = ar br + ai bi,   Im(conj(a) b) = ar bi - ai br
//                 = P1 + P2,                      = P3 - P1 + P2
// with P1 = ar br, P2 = ai bi, P3 = (ar - ai)(br + bi) (Gauss): a 16x16 tile over 4 rows is
// three real MFMAs.  A workgroup owns a chunk of rows of one k-point; it stages 16 rows of all
// 2 nc columns (S and AS) in LDS with coalesced loads, so each column is read from HBM once,
// and its 8 waves share the tiles (wave w and w + 4 run on one SIMD: 5 tiles per SIMD at
// nc <= 64).  Partial tiles per chunk are summed in a fixed order
// afterwards.
// ------------------------------------------------------------------------------------
constexpr int G2_ROWS = 16;
constexpr int G2_COLS = 64;                       // S at [0, 64), AS at [64, 128) of a stage row
constexpr int G2_ZERO = 2 * G2_COLS;              // 16 zero entries (tiles a wave does not own)
constexpr int G2_PITCH = 2 * G2_COLS + 16 + 1;    // LDS row pitch (complex), odd to spread banks
constexpr int G2_WAVES = 8;                       // waves per workgroup of k_gram2
constexpr int G2_THREADS = 64 * G2_WAVES;
constexpr int GW_WAVES = 4;                       // waves per workgroup of k_gramw
constexpr int GW_THREADS = 64 * GW_WAVES;

// MAXT tiles per wave: ceil(ntile / G2_WAVES).  (At nc = 60, 20 tiles over 8 waves leave four
// slots that multiply zeros; 4 waves x 5 tiles would waste none, but at one wave per SIMD it
// measured 45.7 instead of 33 ms per launch.)  COLS: columns a stage row holds per block (64,
// or 96 for the wide blocks of more than 21 columns per k-point).
template <int MAXT, int COLS = G2_COLS>
__global__ __launch_bounds__(G2_THREADS) void k_gram2(const c64* __restrict__ S, const c64* __restrict__ AS, size_t n,
                                               int nc, int kstride, int rows_per_chunk, int ntile,
                                               c64* __restrict__ part, const int* __restrict__ kskip) {
  constexpr int ZERO = 2 * COLS;            // 16 zero entries (tiles a wave does not own)
  constexpr int PITCH = 2 * COLS + 16 + 1;  // LDS row pitch (complex), odd to spread banks
  __shared__ c64 st[G2_ROWS * PITCH];
  const int b = blockIdx.y;
  if (kskip && kskip[b]) return;
  const int chunk = blockIdx.x;
  const int T = (nc + 15) / 16;
  const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
  const int li = lane & 15, lk = lane >> 4;
  // this wave's tiles: t = wave, wave + G2_WAVES, ...; t -> (mat, ti, tj), ti <= tj
  // tiles past nt read the zero entries of the stage rows
  int tmat[MAXT], tti[MAXT], ttj[MAXT];
  for (int t = 0; t < MAXT; ++t) {
    tmat[t] = 1;
    tti[t] = ttj[t] = ZERO / 16;
  }
  int nt = 0;
  {
    int t = 0;
    for (int mat = 0; mat < 2; ++mat)
      for (int i = 0; i < T; ++i)
        for (int j = i; j < T; ++j, ++t)
          if (t % G2_WAVES == wave && nt < MAXT) {
            tmat[nt] = mat;
            tti[nt] = i;
            ttj[nt] = j;
            ++nt;
          }
  }
  // three real products per complex one (Gauss): P1 = Ar Br, P2 = Ai Bi,
  // P3 = (Ar - Ai)(Br + Bi); Re(A^H B) = P1 + P2, Im(A^H B) = P3 - P1 + P2
  d4 p1[MAXT], p2[MAXT], p3[MAXT];
#pragma unroll
  for (int t = 0; t < MAXT; ++t) {
    p1[t] = d4{0, 0, 0, 0};
    p2[t] = d4{0, 0, 0, 0};
    p3[t] = d4{0, 0, 0, 0};
  }
  const c64* Sb = S + (size_t)b * kstride * n;
  const c64* ASb = AS + (size_t)b * kstride * n;
  const size_t r_begin = (size_t)chunk * rows_per_chunk;
  const size_t r_end = std::min(n, r_begin + rows_per_chunk);
  const int ncol2 = 2 * nc;
  constexpr int PER = (G2_ROWS * 2 * COLS + G2_THREADS - 1) / G2_THREADS;  // staged entries per thread
  c64 nxt[PER];
  auto fetch = [&](size_t r0) {
#pragma unroll
    for (int q = 0; q < PER; ++q) {
      const int e = threadIdx.x + q * G2_THREADS;
      c64 v = mk(0.0, 0.0);
      if (e < G2_ROWS * ncol2) {
        const int c = e / G2_ROWS, r = e % G2_ROWS;
        const size_t row = r0 + r;
        if (row < r_end) v = (c < nc) ? Sb[(size_t)c * n + row] : ASb[(size_t)(c - nc) * n + row];
      }
      nxt[q] = v;
    }
  };
  auto stash = [&]() {
#pragma unroll
    for (int q = 0; q < PER; ++q) {
      const int e = threadIdx.x + q * G2_THREADS;
      if (e < G2_ROWS * ncol2) {
        const int c = e / G2_ROWS;
        st[(e % G2_ROWS) * PITCH + (c < nc ? c : COLS + c - nc)] = nxt[q];
      }
    }
  };
  // padding columns (nc..63 of S and of AS) and the zero block stay zero for the whole chunk
  for (int e = threadIdx.x; e < G2_ROWS * PITCH; e += blockDim.x) st[e] = mk(0.0, 0.0);
  __syncthreads();
  if (r_begin < r_end) {
    fetch(r_begin);
    stash();
  }
  __syncthreads();
  // the products of one staged slice for the first K tiles of this wave
  auto multiply = [&](auto kc_) {
    constexpr int K = decltype(kc_)::value;
#pragma unroll
    for (int kb = 0; kb < G2_ROWS; kb += 4) {
      const c64* srow = st + (kb + lk) * PITCH;
      asm volatile("" ::: "memory");  // one 4-row step's operands live at a time (occupancy)
      c64 av[K], bv[K];
#pragma unroll
      for (int t = 0; t < K; ++t) {
        // columns past nc read zeros (the stage is zero-padded)
        const int ca = tti[t] * 16 + li;
        const int cb = ttj[t] * 16 + li;
        av[t] = srow[ca];
        bv[t] = srow[(tmat[t] == 0 ? COLS : 0) + cb];
      }
      // consecutive MFMAs go to different accumulators
#pragma unroll
      for (int t = 0; t < K; ++t) p1[t] = mfma(av[t].re, bv[t].re, p1[t]);
#pragma unroll
      for (int t = 0; t < K; ++t) p2[t] = mfma(av[t].im, bv[t].im, p2[t]);
#pragma unroll
      for (int t = 0; t < K; ++t) p3[t] = mfma(av[t].re - av[t].im, bv[t].re + bv[t].im, p3[t]);
    }
  };
  for (size_t r0 = r_begin; r0 < r_end; r0 += G2_ROWS) {
    const bool more = r0 + G2_ROWS < r_end;
    if (more) fetch(r0 + G2_ROWS);  // next stage in flight while this one is multiplied
    // a wave with a slot to spare skips it (waves w and w + 4 share a SIMD, so at 20 tiles each
    // SIMD multiplies five)
    if constexpr (MAXT > 1) {
      if (nt == MAXT)
        multiply(std::integral_constant<int, MAXT>{});
      else
        multiply(std::integral_constant<int, MAXT - 1>{});
    } else {
      multiply(std::integral_constant<int, MAXT>{});
    }
    __syncthreads();
    if (more) stash();
    __syncthreads();
  }
  // partial tiles: [b][chunk][tile][256], tile id = wave + G2_WAVES t
  const int nchunk = gridDim.x;
#pragma unroll
  for (int t = 0; t < MAXT; ++t) {
    if (t < nt) {
      c64* out = part + (((size_t)b * nchunk + chunk) * ntile + (wave + G2_WAVES * t)) * 256;
#pragma unroll
      for (int r = 0; r < 4; ++r)
        out[(lk + 4 * r) * 16 + li] = mk(p1[t][r] + p2[t][r], p3[t][r] - p1[t][r] + p2[t][r]);
    }
  }
}

// Sum the partial tiles over chunks (fixed order) and scatter: G[mat][b] full nc x nc, lower
// triangle from the conjugate of the upper tiles.
__global__ void k_gram2_reduce(const c64* __restrict__ part, int nchunk, int ntile, int nc, c64* __restrict__ GA,
                               c64* __restrict__ GB, const int* __restrict__ kskip) {
  const int b = blockIdx.z;
  if (kskip && kskip[b]) return;
  const int t = blockIdx.y;
  const int e = threadIdx.x;  // 256 entries of the tile
  const int T = (nc + 15) / 16;
  int mat = 0, ti = 0, tj = 0;
  {
    int c = 0;
    bool found = false;
    for (int m = 0; m < 2 && !found; ++m)
      for (int i = 0; i < T && !found; ++i)
        for (int j = i; j < T && !found; ++j, ++c)
          if (c == t) {
            mat = m;
            ti = i;
            tj = j;
            found = true;
          }
  }
  const c64* src = part + ((size_t)b * nchunk * ntile + t) * 256 + e;
  double sr = 0.0, si = 0.0;
  for (int k = 0; k < nchunk; ++k) {
    const c64 v = src[(size_t)k * ntile * 256];
    sr += v.re;
    si += v.im;
  }
  const int i = ti * 16 + e / 16, j = tj * 16 + e % 16;
  if (i >= nc || j >= nc) return;
  c64* G = (mat == 0 ? GA : GB) + (size_t)b * nc * nc;
  G[(size_t)i * nc + j] = mk(sr, si);
  if (ti != tj) G[(size_t)j * nc + i] = mk(sr, -si);
}

// ------------------------------------------------------------------------------------
// Gram blocks of the new directions only: [GB | GA](:, W) = S^H [W | AW] (nc x 2mb) in one pass
// over S (nc columns) and AW (mb columns); the blocks between X and P follow from the previous
// Rayleigh-Ritz step (X^H X = I, X^H AX = Theta, X^H P = X^H AP = 0, P^H P = I, P^H AP stored by
// it) and are filled by k_gramw_reduce.  Stage row: S at [0, 64), [W | AW] at [64, 64 + 2mb),
// zeros after; the 16x16 tiles (ti < ceil(nc/16), tj < ceil(2mb/16)) are dealt to the waves,
// MAXT = ceil(ntile / GW_WAVES) each (12 tiles at mb = 20: three per wave, none idle).
// ------------------------------------------------------------------------------------
// COLS: columns of S a stage row holds (64, or 96 for blocks of more than 21 columns); WW: room
// for [W | AW] (2mb <= 48, or 64)
template <int MAXT, int COLS = G2_COLS, int WW = 48>
__global__ __launch_bounds__(GW_THREADS) void k_gramw(const c64* __restrict__ S, const c64* __restrict__ AS, size_t n,
                                                      int mb, int kstride, int rows_per_chunk, int ntile,
                                                      c64* __restrict__ part, const int* __restrict__ kskip) {
  constexpr int GW_R = COLS;                 // start of [W | AW] in a stage row
  constexpr int GW_ZERO = COLS + WW;         // 16 zero entries
  constexpr int GW_PITCH = COLS + WW + 16 + 1;
  __shared__ c64 st[G2_ROWS * GW_PITCH];
  const int b = blockIdx.y;
  if (kskip && kskip[b]) return;
  const int nc = 3 * mb;
  const int chunk = blockIdx.x;
  const int TR = (2 * mb + 15) / 16;
  const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
  const int li = lane & 15, lk = lane >> 4;
  int tti[MAXT], ttj[MAXT];
  int nt = 0;
  for (int t = 0; t < MAXT; ++t) {
    const int id = wave + GW_WAVES * t;
    if (id < ntile) {
      tti[t] = id / TR;
      ttj[t] = id % TR;
      ++nt;
    } else {  // reads the zero entries
      tti[t] = GW_ZERO / 16;
      ttj[t] = (GW_ZERO - GW_R) / 16;
    }
  }
  d4 p1[MAXT], p2[MAXT], p3[MAXT];
#pragma unroll
  for (int t = 0; t < MAXT; ++t) {
    p1[t] = d4{0, 0, 0, 0};
    p2[t] = d4{0, 0, 0, 0};
    p3[t] = d4{0, 0, 0, 0};
  }
  const c64* Sb = S + (size_t)b * kstride * n;
  const c64* AWb = AS + ((size_t)b * kstride + mb) * n;
  const size_t r_begin = (size_t)chunk * rows_per_chunk;
  const size_t r_end = std::min(n, r_begin + rows_per_chunk);
  const int ncl = nc + mb;  // loaded columns: S, then AW (at most 4 COLS / 3)
  constexpr int PER = (G2_ROWS * (4 * (COLS / 3)) + GW_THREADS - 1) / GW_THREADS;
  c64 nxt[PER];
  auto fetch = [&](size_t r0) {
#pragma unroll
    for (int q = 0; q < PER; ++q) {
      const int e = threadIdx.x + q * GW_THREADS;
      c64 v = mk(0.0, 0.0);
      if (e < G2_ROWS * ncl) {
        const int c = e / G2_ROWS, r = e % G2_ROWS;
        const size_t row = r0 + r;
        if (row < r_end) v = (c < nc) ? Sb[(size_t)c * n + row] : AWb[(size_t)(c - nc) * n + row];
      }
      nxt[q] = v;
    }
  };
  auto stash = [&]() {
#pragma unroll
    for (int q = 0; q < PER; ++q) {
      const int e = threadIdx.x + q * GW_THREADS;
      if (e < G2_ROWS * ncl) {
        const int c = e / G2_ROWS;
        c64* row = st + (e % G2_ROWS) * GW_PITCH;
        if (c < nc) {
          row[c] = nxt[q];
          if (c >= mb && c < 2 * mb) row[GW_R + c - mb] = nxt[q];  // W, again on the right
        } else {
          row[GW_R + mb + c - nc] = nxt[q];  // AW
        }
      }
    }
  };
  for (int e = threadIdx.x; e < G2_ROWS * GW_PITCH; e += blockDim.x) st[e] = mk(0.0, 0.0);
  __syncthreads();
  if (r_begin < r_end) {
    fetch(r_begin);
    stash();
  }
  __syncthreads();
  for (size_t r0 = r_begin; r0 < r_end; r0 += G2_ROWS) {
    const bool more = r0 + G2_ROWS < r_end;
    if (more) fetch(r0 + G2_ROWS);
#pragma unroll
    for (int kb = 0; kb < G2_ROWS; kb += 4) {
      const c64* srow = st + (kb + lk) * GW_PITCH;
      asm volatile("" ::: "memory");
      c64 av[MAXT], bv[MAXT];
#pragma unroll
      for (int t = 0; t < MAXT; ++t) {
        av[t] = srow[tti[t] * 16 + li];
        bv[t] = srow[GW_R + ttj[t] * 16 + li];
      }
#pragma unroll
      for (int t = 0; t < MAXT; ++t) p1[t] = mfma(av[t].re, bv[t].re, p1[t]);
#pragma unroll
      for (int t = 0; t < MAXT; ++t) p2[t] = mfma(av[t].im, bv[t].im, p2[t]);
#pragma unroll
      for (int t = 0; t < MAXT; ++t) p3[t] = mfma(av[t].re - av[t].im, bv[t].re + bv[t].im, p3[t]);
    }
    __syncthreads();
    if (more) stash();
    __syncthreads();
  }
  const int nchunk = gridDim.x;
#pragma unroll
  for (int t = 0; t < MAXT; ++t) {
    if (t < nt) {
      c64* out = part + (((size_t)b * nchunk + chunk) * ntile + (wave + GW_WAVES * t)) * 256;
#pragma unroll
      for (int r = 0; r < 4; ++r)
        out[(lk + 4 * r) * 16 + li] = mk(p1[t][r] + p2[t][r], p3[t][r] - p1[t][r] + p2[t][r]);
    }
  }
}

// Sum the partial tiles and scatter S^H W into GB(:, W), S^H AW into GA(:, W) (and the
// conjugates into the W rows); blockIdx.y == ntile fills the known X/P blocks instead.
__global__ void k_gramw_reduce(const c64* __restrict__ part, int nchunk, int ntile, int mb, c64* __restrict__ GA,
                               c64* __restrict__ GB, const double* __restrict__ theta,
                               const c64* __restrict__ gapp, const int* __restrict__ kskip) {
  const int b = blockIdx.z;
  if (kskip && kskip[b]) return;
  const int nc = 3 * mb;
  c64* ga = GA + (size_t)b * nc * nc;
  c64* gb = GB + (size_t)b * nc * nc;
  const int t = blockIdx.y;
  if (t == ntile) {
    // X rows/cols are [0, mb), P rows/cols [2mb, 3mb)
    for (int e = threadIdx.x; e < 4 * mb * mb; e += blockDim.x) {
      const int i0 = e / (2 * mb), j0 = e % (2 * mb);
      const int i = i0 < mb ? i0 : i0 + mb, j = j0 < mb ? j0 : j0 + mb;
      const bool xi = i < mb, xj = j < mb;
      c64 vb = mk((i == j) ? 1.0 : 0.0, 0.0), va = mk(0.0, 0.0);
      if (xi && xj) {
        if (i == j) va = mk(theta[b * mb + i], 0.0);
      } else if (!xi && !xj) {
        va = gapp[((size_t)b * mb + (i - 2 * mb)) * mb + (j - 2 * mb)];
      }
      gb[(size_t)i * nc + j] = vb;
      ga[(size_t)i * nc + j] = va;
    }
    return;
  }
  const int e = threadIdx.x;
  const int TR = (2 * mb + 15) / 16;
  const int ti = t / TR, tj = t % TR;
  const c64* src = part + ((size_t)b * nchunk * ntile + t) * 256 + e;
  double sr = 0.0, si = 0.0;
  for (int k = 0; k < nchunk; ++k) {
    const c64 v = src[(size_t)k * ntile * 256];
    sr += v.re;
    si += v.im;
  }
  const int i = ti * 16 + e / 16, jj = tj * 16 + e % 16;
  if (i >= nc || jj >= 2 * mb) return;
  c64* G = (jj < mb) ? gb : ga;
  const int j = mb + (jj < mb ? jj : jj - mb);
  G[(size_t)i * nc + j] = mk(sr, si);
  if (i < mb || i >= 2 * mb) G[(size_t)j * nc + i] = mk(sr, -si);
}

// ------------------------------------------------------------------------------------
// Update: Y_b[:, map(j)] = sum_c S_b[:, c] C_b[c][j], j < q, in place (Y may be S).
// Computed transposed, D = C^T S^T: the B operand lanes read 16 consecutive rows of one
// column (coalesced), the output lanes hold 16 consecutive rows of one output column.
// Re(Y) = Cr Sr - Ci Si, Im(Y) = Cr Si + Ci Sr (three MFMAs per complex product).  Output
// column j goes to column (j < q1 ? ycol0 + j : ycol1 + j - q1).  Each wave owns 16 rows at
// a time, so all reads of its rows happen before its writes and other waves never touch them.
// ------------------------------------------------------------------------------------
// One wave's 16 rows of S_b C_b: the products of all output tiles accumulate in p1, p2, p3
// (Gauss: Re = P1 - P2, Im = P3 - P1 - P2); output lane (lk, li) of tile t holds output column
// t*16 + lk + 4r, r < 4, of row rb*16 + li.  C_b sits zero-padded in LDS (re-read per row
// block so that it does not occupy registers: kept in registers across the loop it would take
// 3/4 of the register file and halve the occupancy).  All 4*PK input loads are issued before
// the MFMAs and are unconditional: the column is clamped below p (those columns meet zero rows
// of the padded C) and the row below n (rows past n are never stored).
// With U (p a multiple of 4) the clamp moves whole groups of 4 columns, so every column offset
// is uniform (scalar registers) and a lane adds only its 32-bit byte offset `boff` (lk*n + row);
// otherwise each lane clamps its own column.
template <int TQ, bool U, int NMAX>
__device__ __forceinline__ void rows_times_c(const c64* Sb, const c64* csh, int p, size_t n, size_t rowc,
                                             uint32_t boff, int lk, int li, d4 (&p1)[TQ], d4 (&p2)[TQ],
                                             d4 (&p3)[TQ]) {
  constexpr int PK = NMAX / 4;
  constexpr int QP = TQ * 16;
  asm volatile("" ::: "memory");
  c64 sv[PK];
  if constexpr (U) {
#pragma unroll
    for (int kb = 0; kb < PK; ++kb) {
      const char* cb = reinterpret_cast<const char*>(Sb + (size_t)min(kb * 4, p - 4) * n);
      sv[kb] = *reinterpret_cast<const c64*>(cb + boff);
    }
  } else {
#pragma unroll
    for (int kb = 0; kb < PK; ++kb) {
      const int c = min(kb * 4 + lk, p - 1);
      sv[kb] = Sb[(size_t)c * n + rowc];
    }
  }
  // keep every load issued ahead of the MFMAs (each MFMA group then waits only for its own)
  asm volatile("" ::: "memory");
#pragma unroll
  for (int t = 0; t < TQ; ++t) {
    p1[t] = d4{0, 0, 0, 0};
    p2[t] = d4{0, 0, 0, 0};
    p3[t] = d4{0, 0, 0, 0};
  }
#pragma unroll
  for (int kb = 0; kb < PK; ++kb) {
    const int ca = kb * 4 + lk;
    // A operand lane (i = li -> output column, k = lk -> input column): C[k][i];
    // B operand lane (k = lk -> input column, j = li -> row): S[row][k]
    c64 cv[TQ];
#pragma unroll
    for (int t = 0; t < TQ; ++t) cv[t] = csh[ca * QP + t * 16 + li];
    const double ssum = sv[kb].re + sv[kb].im;
    // consecutive MFMAs go to different accumulators
#pragma unroll
    for (int t = 0; t < TQ; ++t) p1[t] = mfma(cv[t].re, sv[kb].re, p1[t]);
#pragma unroll
    for (int t = 0; t < TQ; ++t) p2[t] = mfma(cv[t].im, sv[kb].im, p2[t]);
#pragma unroll
    for (int t = 0; t < TQ; ++t) p3[t] = mfma(cv[t].re + cv[t].im, ssum, p3[t]);
  }
}

// Element (column col, lane offset) of a column block: with U the column part is uniform and
// the lane part is the 32-bit byte offset boff, else plain indexing with the lane's row.
template <bool U>
__device__ __forceinline__ c64& elem(c64* base, int col, size_t n, uint32_t boff, size_t row) {
  if constexpr (U)
    return *reinterpret_cast<c64*>(reinterpret_cast<char*>(base + (size_t)col * n) + boff);
  else
    return base[(size_t)col * n + row];
}

// C_b (p x q) into LDS, zero-padded to NMAX x TQ*16
template <int TQ, int NMAX>
__device__ __forceinline__ void stage_c(const c64* Cb, c64* csh, int p, int q) {
  constexpr int QP = TQ * 16;
  for (int t = threadIdx.x; t < NMAX * QP; t += blockDim.x) {
    const int r = t / QP, c = t % QP;
    csh[t] = (r < p && c < q) ? Cb[r * q + c] : mk(0.0, 0.0);
  }
}

template <int TQ, bool U, int NMAX = RR_NMAX>
__global__ __launch_bounds__(256) void k_update(const c64* S, c64* Y, const c64* __restrict__ C, size_t n,
                                                int p, int q, int skstride, int scol0, int ykstride, int q1,
                                                int ycol0, int ycol1, const int* __restrict__ kskip) {
  extern __shared__ c64 csh[];  // C_b zero-padded to NMAX x TQ*16
  const int b = blockIdx.y;
  if (kskip && kskip[b]) return;
  stage_c<TQ, NMAX>(C + (size_t)b * p * q, csh, p, q);
  __syncthreads();
  const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
  const int li = lane & 15, lk = lane >> 4;
  const c64* Sb = S + ((size_t)b * skstride + scol0) * n;
  c64* Yb = Y + (size_t)b * ykstride * n;
  const int ucol = U ? 0 : 1;  // with U (p, q, q1 multiples of 4) the lane's lk is in boff
  const size_t nblk = (n + 15) / 16;
  for (size_t rb = (size_t)blockIdx.x * 4 + wave; rb < nblk; rb += (size_t)gridDim.x * 4) {
    const size_t row = rb * 16 + li;
    const bool rok = row < n;
    const size_t rowc = rok ? row : n - 1;
    const uint32_t boff = (uint32_t)(((size_t)lk * n + rowc) * sizeof(c64));
    d4 p1[TQ], p2[TQ], p3[TQ];
    rows_times_c<TQ, U, NMAX>(Sb, csh, p, n, rowc, boff, lk, li, p1, p2, p3);
#pragma unroll
    for (int t = 0; t < TQ; ++t)
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        const int j = t * 16 + lk + 4 * r, ju = t * 16 + 4 * r + lk * ucol;
        if (rok && j < q)
          elem<U>(Yb, (ju < q1) ? ycol0 + ju : ycol1 + (ju - q1), n, boff, row) =
              mk(p1[t][r] - p2[t][r], p3[t][r] - p1[t][r] - p2[t][r]);
      }
  }
}

// The two block updates of a Rayleigh-Ritz step in one pass, with the next residuals:
// [X P] <- S [C1 Cp] and [AX AP] <- AS [C1 Cp] in place (S = [X W P] and AS as kstride-spaced
// groups of 3mb columns; X to columns 0..mb-1, P to 2mb..3mb-1), then from the new X and AX of
// the same 16 rows, still in registers, R_j = AX_j - theta_j X_j (eq (4.3)) into the contiguous
// R ([b*mb + j][n]) and per-workgroup partial sums of |r_j|^2 and |x_j|^2 (part, the layout of
// k_resid_reduce).  X column j = 4s + lk is slot s < XS of lane (lk, li): tile s/4, entry s%4;
// between the two products each lane parks its new X values in a private LDS slot (in registers
// they would push the kernel to one wave per SIMD).
template <int XS, bool U, int NMAX = RR_NMAX>
__global__ __launch_bounds__(256) void k_update_res(c64* S, c64* AS, const c64* __restrict__ C, size_t n, int mb,
                                                    int kstride, const double* __restrict__ theta,
                                                    c64* __restrict__ R, double* __restrict__ part,
                                                    const int* __restrict__ kskip) {
  constexpr int TQ = (XS + 1) / 2;  // 2mb output columns in tiles of 16
  extern __shared__ c64 csh[];  // C_b (NMAX x TQ*16), then the parked X values [4][XS][64]
  __shared__ double th[NMAX / 3];
  __shared__ double red[4][XS][4][2];
  c64* xpark = csh + NMAX * TQ * 16;
  const int b = blockIdx.y;
  if (kskip && kskip[b]) return;
  const int p = 3 * mb, q = 2 * mb;
  stage_c<TQ, NMAX>(C + (size_t)b * p * q, csh, p, q);
  for (int j = threadIdx.x; j < mb; j += blockDim.x) th[j] = theta[b * mb + j];
  __syncthreads();
  const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
  const int li = lane & 15, lk = lane >> 4;
  c64* Sb = S + (size_t)b * kstride * n;
  c64* ASb = AS + (size_t)b * kstride * n;
  c64* Rb = R + (size_t)b * mb * n;
  // with U, output column t*16 + lk + 4r is column t*16 + 4r of the lane's base (lk*n + row),
  // and which of X / P it belongs to does not depend on lk (mb is a multiple of 4)
  const int ucol = U ? 0 : 1;
  double rr[XS], xx[XS];
#pragma unroll
  for (int s = 0; s < XS; ++s) rr[s] = xx[s] = 0.0;
  const size_t nblk = (n + 15) / 16;
  for (size_t rb = (size_t)blockIdx.x * 4 + wave; rb < nblk; rb += (size_t)gridDim.x * 4) {
    const size_t row = rb * 16 + li;
    const bool rok = row < n;
    const size_t rowc = rok ? row : n - 1;
    const uint32_t boff = (uint32_t)(((size_t)lk * n + rowc) * sizeof(c64));
    c64* xk = xpark + (size_t)wave * XS * 64 + lane;  // slot s at xk[s * 64]
    {
      d4 p1[TQ], p2[TQ], p3[TQ];
      rows_times_c<TQ, U, NMAX>(Sb, csh, p, n, rowc, boff, lk, li, p1, p2, p3);
#pragma unroll
      for (int t = 0; t < TQ; ++t)
#pragma unroll
        for (int r = 0; r < 4; ++r) {
          const int j = t * 16 + lk + 4 * r, ju = t * 16 + 4 * r + lk * ucol;
          const c64 v = mk(p1[t][r] - p2[t][r], p3[t][r] - p1[t][r] - p2[t][r]);
          if (t * 4 + r < XS) xk[(t * 4 + r) * 64] = v;
          if (rok && j < q) elem<U>(Sb, ju < mb ? ju : mb + ju, n, boff, row) = v;
        }
    }
    {
      d4 p1[TQ], p2[TQ], p3[TQ];
      rows_times_c<TQ, U, NMAX>(ASb, csh, p, n, rowc, boff, lk, li, p1, p2, p3);
#pragma unroll
      for (int t = 0; t < TQ; ++t)
#pragma unroll
        for (int r = 0; r < 4; ++r) {
          const int j = t * 16 + lk + 4 * r, ju = t * 16 + 4 * r + lk * ucol;
          const c64 v = mk(p1[t][r] - p2[t][r], p3[t][r] - p1[t][r] - p2[t][r]);
          if (rok && j < q) elem<U>(ASb, ju < mb ? ju : mb + ju, n, boff, row) = v;
          if (t * 4 + r < XS) {
            const int s = t * 4 + r;
            if (rok && j < mb) {
              const c64 x = xk[s * 64];
              const c64 rv = v - th[j] * x;
              elem<U>(Rb, ju, n, boff, row) = rv;
              rr[s] += abs2(rv);
              xx[s] += abs2(x);
            }
          }
        }
    }
  }
  // sums over the 16 rows of a lane group (li), then over the waves, in a fixed order
#pragma unroll
  for (int s = 0; s < XS; ++s)
#pragma unroll
    for (int o = 8; o > 0; o >>= 1) {
      rr[s] += __shfl_xor(rr[s], o, 16);
      xx[s] += __shfl_xor(xx[s], o, 16);
    }
  if (li == 0)
#pragma unroll
    for (int s = 0; s < XS; ++s) {
      red[wave][s][lk][0] = rr[s];
      red[wave][s][lk][1] = xx[s];
    }
  __syncthreads();
  if ((int)threadIdx.x < 2 * mb) {
    const int j = threadIdx.x >> 1, c = threadIdx.x & 1;
    const double v = red[0][j >> 2][j & 3][c] + red[1][j >> 2][j & 3][c] + red[2][j >> 2][j & 3][c] +
                     red[3][j >> 2][j & 3][c];
    part[(((size_t)b * mb + j) * gridDim.x + blockIdx.x) * 2 + c] = v;
  }
}

// ------------------------------------------------------------------------------------
// Residual + preconditioner: r_j = AX_j - theta_j X_j, W_j = K_P^{-1} r_j (closed form of
// the diagonal-block preconditioner, eqs (2.31)-(2.32)), per-block partial sums of |r_j|^2
// and |x_j|^2; optionally a contiguous copy of r (Rout, [b*mb + j][3N^3]); W is not written
// for the k-points whose wskip is set (their new directions come from another preconditioner).
// Grid: x = blocks per vector, y = column j, z = k-point b.
// ------------------------------------------------------------------------------------
__global__ __launch_bounds__(256) void k_resid_precond(const c64* __restrict__ S, const c64* __restrict__ AS,
                                                       c64* __restrict__ Wout, const double* __restrict__ theta,
                                                       const c64* __restrict__ ktab64,
                                                       const double* __restrict__ gamma, int N, int kstride,
                                                       int xcol0, int wcol0, int mb, double* __restrict__ part,
                                                       const int* __restrict__ kskip, c64* __restrict__ Rout,
                                                       const int* __restrict__ wskip,
                                                       const double* __restrict__ sfl, Skew sk) {
  const int b = blockIdx.z, j = blockIdx.y;
  if (kskip && kskip[b]) return;
  const bool ww = !(wskip && wskip[b]);
  const size_t N3 = (size_t)N * N * N, n = 3 * N3;
  const c64* x = S + ((size_t)b * kstride + xcol0 + j) * n;
  const c64* ax = AS + ((size_t)b * kstride + xcol0 + j) * n;
  c64* w = Wout + ((size_t)b * kstride + wcol0 + j) * n;
  const double th = theta[b * mb + j];
  const c64* K = ktab64 + (size_t)b * 3 * N;
  const double g = gamma[b];
  const double fl = sfl ? sfl[b] : 0.0;
  c64* rc = Rout ? Rout + ((size_t)b * mb + j) * n : nullptr;
  double rr = 0.0, xx = 0.0;
  for (size_t p = (size_t)blockIdx.x * blockDim.x + threadIdx.x; p < N3; p += (size_t)gridDim.x * blockDim.x) {
    const int qx = (int)(p % N), qy = (int)((p / N) % N), qz = (int)(p / ((size_t)N * N));
    c64 K1 = K[qx], K2 = K[N + qy], K3 = K[2 * N + qz];
    skew_fix<double>(sk, qx, qy, qz, K1, K2, K3);
    const c64 x1 = x[p], x2 = x[N3 + p], x3 = x[2 * N3 + p];
    const c64 r1 = ax[p] - th * x1, r2 = ax[N3 + p] - th * x2, r3 = ax[2 * N3 + p] - th * x3;
    rr += abs2(r1) + abs2(r2) + abs2(r3);
    xx += abs2(x1) + abs2(x2) + abs2(x3);
    const double s = abs2(K1) + abs2(K2) + abs2(K3);
    c64 w1 = mk(0.0, 0.0), w2 = w1, w3 = w1;
    if (s != 0.0) {
      // 1/s on the transverse and 1/(gamma s) on the longitudinal part, with s floored at fl
      // (the floor bounds the gain near k = 0, where s at the DC frequency is |k|^2)
      const double is = 1.0 / s, ie = s < fl ? 1.0 / fl : is;
      const c64 u = ((1.0 / g - 1.0) * ie * is) * (K1 * r1 + K2 * r2 + K3 * r3);
      w1 = ie * r1 + cmulc(K1, u);
      w2 = ie * r2 + cmulc(K2, u);
      w3 = ie * r3 + cmulc(K3, u);
    }
    if (ww) {
      w[p] = w1;
      w[N3 + p] = w2;
      w[2 * N3 + p] = w3;
    }
    if (rc) {
      rc[p] = r1;
      rc[N3 + p] = r2;
      rc[2 * N3 + p] = r3;
    }
  }
  // block reduction (fixed order)
  __shared__ double sr[256], sx[256];
  sr[threadIdx.x] = rr;
  sx[threadIdx.x] = xx;
  __syncthreads();
  for (int o = 128; o > 0; o >>= 1) {
    if ((int)threadIdx.x < o) {
      sr[threadIdx.x] += sr[threadIdx.x + o];
      sx[threadIdx.x] += sx[threadIdx.x + o];
    }
    __syncthreads();
  }
  if (threadIdx.x == 0) {
    double* o = part + (((size_t)b * mb + j) * gridDim.x + blockIdx.x) * 2;
    o[0] = sr[0];
    o[1] = sx[0];
  }
}

// ------------------------------------------------------------------------------------
// Deflation of the DC longitudinal direction for the k-points with dcl[b] != 0: at the
// frequency p = 0, x(0) <- x(0) - conj(K(0)) (K(0) . x(0)) / |K(0)|^2.  That direction (the
// constant field along k) is an eigenvector of Op with eigenvalue gamma |k|^2 (Prop 2.3).
// Columns [col0, col0 + ncol) of each k-point's group (kstride-spaced); one thread per column.
// ------------------------------------------------------------------------------------
__global__ void k_deflate_dc_long(c64* __restrict__ S, int kstride, int col0, int ncol, int nb,
                                  const c64* __restrict__ ktab64, int N, const int* __restrict__ dcl) {
  const int t = blockIdx.x * blockDim.x + threadIdx.x;
  if (t >= nb * ncol) return;
  const int b = t / ncol, j = t % ncol;
  if (!dcl[b]) return;
  const size_t N3 = (size_t)N * N * N;
  c64* x = S + ((size_t)b * kstride + col0 + j) * 3 * N3;
  const c64* K = ktab64 + (size_t)b * 3 * N;
  const c64 K1 = K[0], K2 = K[N], K3 = K[2 * N];
  const double s = abs2(K1) + abs2(K2) + abs2(K3);
  if (s == 0.0) return;
  const c64 x1 = x[0], x2 = x[N3], x3 = x[2 * N3];
  const c64 u = (1.0 / s) * (K1 * x1 + K2 * x2 + K3 * x3);
  x[0] = x1 - cmulc(K1, u);
  x[N3] = x2 - cmulc(K2, u);
  x[2 * N3] = x3 - cmulc(K3, u);
}

int deflate_dc_long(c64* S, int kstride, int col0, int ncol, int nb, const c64* ktab64, int N, const int* dcl,
                    hipStream_t s) {
  const int tot = nb * ncol;
  k_deflate_dc_long<<<(tot + 255) / 256, 256, 0, s>>>(S, kstride, col0, ncol, nb, ktab64, N, dcl);
  KC_LAUNCHED();
  return KC_OK;
}

__global__ void k_resid_reduce(const double* __restrict__ part, int nblk, int nvec, double* __restrict__ res,
                               double* __restrict__ xnorm2, double* __restrict__ rnorm2) {
  const int v = blockIdx.x * blockDim.x + threadIdx.x;
  if (v >= nvec) return;
  double a = 0.0, c = 0.0;
  for (int i = 0; i < nblk; ++i) {
    a += part[((size_t)v * nblk + i) * 2];
    c += part[((size_t)v * nblk + i) * 2 + 1];
  }
  res[v] = (c > 0.0) ? sqrt(a / c) : 0.0;
  if (xnorm2) xnorm2[v] = c;
  if (rnorm2) rnorm2[v] = a;
}

// ------------------------------------------------------------------------------------
// Seeded initial block: entries uniform in [-1/2, 1/2) (real and imaginary parts) from a
// counter-based generator (the splitmix64 finaliser applied to a unique 64-bit counter).
// ------------------------------------------------------------------------------------
__device__ __forceinline__ uint64_t mix64(uint64_t z) {
  z += 0x9E3779B97F4A7C15ull;
  z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
  z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
  return z ^ (z >> 31);
}

__global__ void k_random_block(c64* S, size_t n, int kstride, int col0, int ncol, uint64_t seed,
                               const int* __restrict__ kglobal) {
  const int b = blockIdx.z, j = blockIdx.y;
  if (j >= ncol) return;
  c64* v = S + ((size_t)b * kstride + col0 + j) * n;
  const uint64_t base = mix64(seed ^ mix64(((uint64_t)kglobal[b] << 20) ^ (uint64_t)j));
  for (size_t p = (size_t)blockIdx.x * blockDim.x + threadIdx.x; p < n; p += (size_t)gridDim.x * blockDim.x) {
    const uint64_t h = mix64(base + 2 * p), g = mix64(base + 2 * p + 1);
    const double r = (double)(h >> 11) * (1.0 / 9007199254740992.0) - 0.5;
    const double i = (double)(g >> 11) * (1.0 / 9007199254740992.0) - 0.5;
    v[p] = mk(r, i);
  }
}

// column j of k-point b: the plane wave with frequency q[b][j] (flattened, x fastest) and
// polarization pol[b][j][3], zero elsewhere; q < 0 leaves the column as it is
__global__ void k_plane_waves(c64* S, size_t n, size_t N3, int kstride, int col0, int ncol, const int* __restrict__ q,
                              const c64* __restrict__ pol) {
  const int b = blockIdx.z, j = blockIdx.y;
  c64* v = S + ((size_t)b * kstride + col0 + j) * n;
  if (q[b * ncol + j] < 0) return;
  const size_t qq = (size_t)q[b * ncol + j];
  const c64* pp = pol + ((size_t)b * ncol + j) * 3;
  for (size_t t = (size_t)blockIdx.x * blockDim.x + threadIdx.x; t < n; t += (size_t)gridDim.x * blockDim.x) {
    const size_t c = t / N3, p = t - c * N3;
    v[t] = (p == qq) ? pp[c] : mk(0.0, 0.0);
  }
}

// ------------------------------------------------------------------------------------
// host launchers
// ------------------------------------------------------------------------------------
// rows per workgroup of the Gram kernels (a multiple of G2_ROWS, about 2048 workgroups in all)
static size_t gram_rows(size_t n, int nb) {
  const size_t target_wg = 2048;
  const size_t per_k = std::max<size_t>(1, target_wg / (size_t)nb);
  size_t rows = (n + per_k - 1) / per_k;
  rows = std::max<size_t>(rows, 64);
  return (rows + G2_ROWS - 1) / G2_ROWS * G2_ROWS;
}

size_t gram2_part_bytes(int nc, size_t n, int nb) {
  const int T = (nc + 15) / 16;
  const size_t rows = gram_rows(n, nb);
  return (size_t)nb * ((n + rows - 1) / rows) * (T * (T + 1)) * 256 * sizeof(c64);
}

// gram2 with the rows of a chunk given (a multiple of G2_ROWS)
static int gram2_rows(const c64* S, const c64* AS, int kstride, int nc, size_t n, int nb, c64* part, c64* GA,
                      c64* GB, const int* kskip, size_t rows, hipStream_t s);

int gram2(const c64* S, const c64* AS, int kstride, int nc, size_t n, int nb, c64* part, c64* GA, c64* GB,
          const int* kskip, hipStream_t s) {
  return gram2_rows(S, AS, kstride, nc, n, nb, part, GA, GB, kskip, gram_rows(n, nb), s);
}

int gram2_bounded(const c64* S, const c64* AS, int nc, size_t n, int nb, c64* part, size_t part_bytes, c64* GA,
                  c64* GB, hipStream_t s) {
  const int T = (nc + 15) / 16;
  const size_t per_chunk = (size_t)nb * (T * (T + 1)) * 256 * sizeof(c64);  // one chunk per k-point
  if (per_chunk > part_bytes) {
    set_error("gram2: partial sums of " + std::to_string(nb) + " k-points exceed the " + std::to_string(part_bytes) +
              "-byte buffer");
    return KC_ERR_INVALID_ARG;
  }
  const size_t max_chunks = part_bytes / per_chunk;
  size_t rows = gram_rows(n, nb);
  if ((n + rows - 1) / rows > max_chunks) {
    rows = (n + max_chunks - 1) / max_chunks;
    rows = (rows + G2_ROWS - 1) / G2_ROWS * G2_ROWS;
  }
  if (rows > (size_t)INT32_MAX) {
    set_error("gram2: too many rows per chunk");
    return KC_ERR_INVALID_ARG;
  }
  return gram2_rows(S, AS, nc, nc, n, nb, part, GA, GB, nullptr, rows, s);
}

static int gram2_rows(const c64* S, const c64* AS, int kstride, int nc, size_t n, int nb, c64* part, c64* GA,
                      c64* GB, const int* kskip, size_t rows, hipStream_t s) {
  const int T = (nc + 15) / 16;
  const int ntile = T * (T + 1);
  if (nc > RR_NMAX_WIDE) {
    set_error("gram2: too many columns");
    return KC_ERR_INVALID_ARG;
  }
  const int nchunk = (int)((n + rows - 1) / rows);
  dim3 grid(nchunk, nb);
  if (nc <= G2_COLS) {
    switch ((ntile + G2_WAVES - 1) / G2_WAVES) {
      case 1: k_gram2<1><<<grid, G2_THREADS, 0, s>>>(S, AS, n, nc, kstride, (int)rows, ntile, part, kskip); break;
      case 2: k_gram2<2><<<grid, G2_THREADS, 0, s>>>(S, AS, n, nc, kstride, (int)rows, ntile, part, kskip); break;
      default: k_gram2<3><<<grid, G2_THREADS, 0, s>>>(S, AS, n, nc, kstride, (int)rows, ntile, part, kskip); break;
    }
  } else if (nc <= 80) {  // 65..80 columns: 30 tiles on an 80-column stage
    k_gram2<4, 80><<<grid, G2_THREADS, 0, s>>>(S, AS, n, nc, kstride, (int)rows, ntile, part, kskip);
  } else {  // 81..96 columns: 42 tiles
    k_gram2<6, RR_NMAX_WIDE><<<grid, G2_THREADS, 0, s>>>(S, AS, n, nc, kstride, (int)rows, ntile, part, kskip);
  }
  KC_LAUNCHED();
  dim3 g2(1, ntile, nb);
  k_gram2_reduce<<<g2, 256, 0, s>>>(part, nchunk, ntile, nc, GA, GB, kskip);
  KC_LAUNCHED();
  return KC_OK;
}

int gram2(const c64* S, const c64* AS, int kstride, int nc, size_t n, int nb, DevBuf& part, c64* GA, c64* GB,
          const int* kskip, hipStream_t s) {
  KC_TRY(part.ensure(gram2_part_bytes(nc, n, nb)));
  return gram2(S, AS, kstride, nc, n, nb, part.as<c64>(), GA, GB, kskip, s);
}

int gramw(const c64* S, const c64* AS, int kstride, int mb, size_t n, int nb, DevBuf& part, c64* GA, c64* GB,
          const double* theta, const c64* gapp, const int* kskip, hipStream_t s) {
  const int nc = 3 * mb;
  const int T = (nc + 15) / 16, TR = (2 * mb + 15) / 16;
  const int ntile = T * TR;
  if (nc > RR_NMAX_WIDE) {
    set_error("gramw: too many columns");
    return KC_ERR_INVALID_ARG;
  }
  const size_t rows = gram_rows(n, nb);
  const int nchunk = (int)((n + rows - 1) / rows);
  KC_TRY(part.ensure((size_t)nb * nchunk * ntile * 256 * sizeof(c64)));
  dim3 grid(nchunk, nb);
  c64* pp = part.as<c64>();
  const int maxt = (ntile + GW_WAVES - 1) / GW_WAVES;
  if (nc <= G2_COLS && 2 * mb <= 48) {  // at most 16 tiles
    switch (maxt) {
      case 1: k_gramw<1><<<grid, GW_THREADS, 0, s>>>(S, AS, n, mb, kstride, (int)rows, ntile, pp, kskip); break;
      case 2: k_gramw<2><<<grid, GW_THREADS, 0, s>>>(S, AS, n, mb, kstride, (int)rows, ntile, pp, kskip); break;
      default: k_gramw<3><<<grid, GW_THREADS, 0, s>>>(S, AS, n, mb, kstride, (int)rows, ntile, pp, kskip); break;
    }
  } else {  // the wide blocks: up to 6 x 4 tiles
    switch (maxt) {
      case 4: k_gramw<4, 96, 64><<<grid, GW_THREADS, 0, s>>>(S, AS, n, mb, kstride, (int)rows, ntile, pp, kskip); break;
      case 5: k_gramw<5, 96, 64><<<grid, GW_THREADS, 0, s>>>(S, AS, n, mb, kstride, (int)rows, ntile, pp, kskip); break;
      default: k_gramw<6, 96, 64><<<grid, GW_THREADS, 0, s>>>(S, AS, n, mb, kstride, (int)rows, ntile, pp, kskip); break;
    }
  }
  KC_LAUNCHED();
  dim3 g2(1, ntile + 1, nb);
  k_gramw_reduce<<<g2, 256, 0, s>>>(part.as<c64>(), nchunk, ntile, mb, GA, GB, theta, gapp, kskip);
  KC_LAUNCHED();
  return KC_OK;
}

// rows of C staged by the update kernels of the wide path: 3mb rounded up to 72, 84 or 96, so
// that no k-step multiplies only padding (and at mb <= 24 two workgroups fit a CU's LDS)
static int wide_rows(int p) { return p <= 72 ? 72 : p <= 84 ? 84 : RR_NMAX_WIDE; }

int update(const c64* S, int skstride, int scol0, int p, c64* Y, int ykstride, int q, int q1, int ycol0,
           int ycol1, const c64* C, size_t n, int nb, const int* kskip, hipStream_t s) {
  dim3 grid(update_grid_x(n, nb), nb);
  if (p > RR_NMAX_WIDE || q > 64) {
    set_error("update: too many input or output columns");
    return KC_ERR_INVALID_ARG;
  }
  const bool wide = p > RR_NMAX;
  const int rows = wide ? wide_rows(p) : RR_NMAX;
  const size_t shm = (size_t)rows * ((q + 15) / 16 * 16) * sizeof(c64);
  const bool u = p % 4 == 0 && q % 4 == 0 && q1 % 4 == 0 && 4 * n * sizeof(c64) < (size_t(1) << 32);
#define KC_UPD(T, NM)                                                                                        \
  if (u)                                                                                                     \
    k_update<T, true, NM><<<grid, 256, shm, s>>>(S, Y, C, n, p, q, skstride, scol0, ykstride, q1, ycol0, ycol1, \
                                                 kskip);                                                     \
  else                                                                                                       \
    k_update<T, false, NM><<<grid, 256, shm, s>>>(S, Y, C, n, p, q, skstride, scol0, ykstride, q1, ycol0,    \
                                                  ycol1, kskip)
  if (wide) {
    // the wide path (more than 21 columns per block): C needs more than 64 KiB of LDS
    KC_TRY(update_res_prepare());
    if (rows == 72) {
      if (q <= 48) {
        KC_UPD(3, 72);
      } else {
        KC_UPD(4, 72);
      }
    } else if (rows == 84) {
      if (q <= 48) {
        KC_UPD(3, 84);
      } else {
        KC_UPD(4, 84);
      }
    } else if (q <= 48) {
      KC_UPD(3, 96);
    } else {
      KC_UPD(4, 96);
    }
  } else if (q <= 16) {
    KC_UPD(1, RR_NMAX);
  } else if (q <= 32) {
    KC_UPD(2, RR_NMAX);
  } else if (q <= 48) {
    KC_UPD(3, RR_NMAX);
  } else {
    set_error("update: too many output columns");
    return KC_ERR_INVALID_ARG;
  }
#undef KC_UPD
  KC_LAUNCHED();
  return KC_OK;
}

unsigned update_grid_x(size_t n, int nb) {
  const size_t nblk = (n + 15) / 16;
  return (unsigned)std::max<size_t>(1, std::min<size_t>((nblk + 3) / 4, 4096 / std::max(nb, 1) + 1));
}

// dynamic LDS of k_update_res: C_b and the parked X values
static size_t update_res_lds_n(int xs, int nmax) {
  return ((size_t)nmax * (((xs + 1) / 2) * 16) + (size_t)4 * xs * 64) * sizeof(c64);
}
// rows of C staged for mb columns: 60 at 17..20 (the bench's 16 + 4), RR_NMAX up to 21, then
// the wide rows
static int update_res_rows(int mb) {
  return 3 * mb > RR_NMAX ? wide_rows(3 * mb) : (mb >= 17 && mb <= 20) ? 60 : RR_NMAX;
}
static size_t update_res_lds(int mb) { return update_res_lds_n((mb + 3) / 4, update_res_rows(mb)); }

int update_res_prepare() {
  static bool done = false;
  if (done) return KC_OK;
  const void* k[12] = {(const void*)k_update_res<1, false>, (const void*)k_update_res<2, false>,
                       (const void*)k_update_res<3, false>, (const void*)k_update_res<4, false>,
                       (const void*)k_update_res<5, false>, (const void*)k_update_res<6, false>,
                       (const void*)k_update_res<1, true>,  (const void*)k_update_res<2, true>,
                       (const void*)k_update_res<3, true>,  (const void*)k_update_res<4, true>,
                       (const void*)k_update_res<5, true>,  (const void*)k_update_res<6, true>};
  for (int i = 0; i < 12; ++i)
    KC_HIP(hipFuncSetAttribute(k[i], hipFuncAttributeMaxDynamicSharedMemorySize,
                               (int)update_res_lds_n(i % 6 + 1, RR_NMAX)));
  // 17..20 columns per block: C staged at 60 rows (no k-step of padding only)
  KC_HIP(hipFuncSetAttribute((const void*)k_update_res<5, false, 60>, hipFuncAttributeMaxDynamicSharedMemorySize,
                             (int)update_res_lds(20)));
  KC_HIP(hipFuncSetAttribute((const void*)k_update_res<5, true, 60>, hipFuncAttributeMaxDynamicSharedMemorySize,
                             (int)update_res_lds(20)));
  // the wide path: 22 <= mb <= 32 (xs 6..8 with 72, 84, 96 staged rows of C), and the plain
  // update with up to 96 input and 64 output columns
  const void* kw[6] = {(const void*)k_update_res<6, false, 72>, (const void*)k_update_res<7, false, 84>,
                       (const void*)k_update_res<8, false, 96>, (const void*)k_update_res<6, true, 72>,
                       (const void*)k_update_res<7, true, 84>,  (const void*)k_update_res<8, true, 96>};
  const int kwmb[6] = {24, 28, 32, 24, 28, 32};
  for (int i = 0; i < 6; ++i)
    KC_HIP(hipFuncSetAttribute(kw[i], hipFuncAttributeMaxDynamicSharedMemorySize, (int)update_res_lds(kwmb[i])));
  const void* ku[12] = {(const void*)k_update<3, false, 72>, (const void*)k_update<4, false, 72>,
                        (const void*)k_update<3, true, 72>,  (const void*)k_update<4, true, 72>,
                        (const void*)k_update<3, false, 84>, (const void*)k_update<4, false, 84>,
                        (const void*)k_update<3, true, 84>,  (const void*)k_update<4, true, 84>,
                        (const void*)k_update<3, false, 96>, (const void*)k_update<4, false, 96>,
                        (const void*)k_update<3, true, 96>,  (const void*)k_update<4, true, 96>};
  const int kur[3] = {72, 84, 96};
  for (int i = 0; i < 12; ++i)
    KC_HIP(hipFuncSetAttribute(ku[i], hipFuncAttributeMaxDynamicSharedMemorySize,
                               (int)(kur[i / 4] * 64 * sizeof(c64))));
  done = true;
  return KC_OK;
}

int update_res(c64* S, c64* AS, int kstride, int mb, const c64* C, size_t n, int nb, const double* theta, c64* R,
               double* part, double* res, double* xnorm2, const int* kskip, hipStream_t s) {
  if (mb < 1 || 3 * mb > RR_NMAX_WIDE) {
    set_error("update_res: block size out of range");
    return KC_ERR_INVALID_ARG;
  }
  const unsigned gx = update_grid_x(n, nb);
  dim3 grid(gx, nb);
  const int xs = (mb + 3) / 4;
  const size_t shm = update_res_lds(mb);
  // uniform column offsets need whole groups of 4 columns and 32-bit lane byte offsets
  const bool u = (mb % 4 == 0) && 4 * n * sizeof(c64) < (size_t(1) << 32);
#define KC_UPDRES(X)                                                                          \
  if (u)                                                                                      \
    k_update_res<X, true><<<grid, 256, shm, s>>>(S, AS, C, n, mb, kstride, theta, R, part, kskip); \
  else                                                                                        \
    k_update_res<X, false><<<grid, 256, shm, s>>>(S, AS, C, n, mb, kstride, theta, R, part, kskip)
#define KC_UPDRES_W(X, NM)                                                                    \
  if (u)                                                                                      \
    k_update_res<X, true, NM><<<grid, 256, shm, s>>>(S, AS, C, n, mb, kstride, theta, R, part, kskip); \
  else                                                                                        \
    k_update_res<X, false, NM><<<grid, 256, shm, s>>>(S, AS, C, n, mb, kstride, theta, R, part, kskip)
  if (3 * mb > RR_NMAX) {
    // xs 6, 7, 8 <-> mb 22..24, 25..28, 29..32 <-> 72, 84, 96 staged rows
    KC_TRY(update_res_prepare());
    switch (xs) {
      case 6: KC_UPDRES_W(6, 72); break;
      case 7: KC_UPDRES_W(7, 84); break;
      default: KC_UPDRES_W(8, 96); break;
    }
  } else switch (xs) {
    case 1: KC_UPDRES(1); break;
    case 2: KC_UPDRES(2); break;
    case 3: KC_UPDRES(3); break;
    case 4: KC_UPDRES(4); break;
    case 5: KC_UPDRES_W(5, 60); break;  // mb 17..20
    default: KC_UPDRES(6); break;
  }
#undef KC_UPDRES
#undef KC_UPDRES_W
  KC_LAUNCHED();
  const int nv = nb * mb;
  k_resid_reduce<<<(nv + 255) / 256, 256, 0, s>>>(part, (int)gx, nv, res, xnorm2, nullptr);
  KC_LAUNCHED();
  return KC_OK;
}

int resid_precond(const c64* S, const c64* AS, c64* W, const double* theta, const c64* ktab64,
                  const double* gamma, int N, int kstride, int xcol0, int wcol0, int mb, int nb, DevBuf& part,
                  double* res, double* xnorm2, const int* kskip, hipStream_t s, c64* Rout, double* rnorm2,
                  const int* wskip, const double* sfl, const Skew* sk) {
  const size_t N3 = (size_t)N * N * N;
  const int nblk = (int)std::max<size_t>(1, std::min<size_t>((N3 + 255) / 256, 256));
  KC_TRY(part.ensure((size_t)nb * mb * nblk * 2 * sizeof(double)));
  dim3 grid(nblk, mb, nb);
  k_resid_precond<<<grid, 256, 0, s>>>(S, AS, W, theta, ktab64, gamma, N, kstride, xcol0, wcol0, mb,
                                       part.as<double>(), kskip, Rout, wskip, sfl, sk ? *sk : Skew());
  KC_LAUNCHED();
  const int nv = nb * mb;
  k_resid_reduce<<<(nv + 255) / 256, 256, 0, s>>>(part.as<double>(), nblk, nv, res, xnorm2, rnorm2);
  KC_LAUNCHED();
  return KC_OK;
}

int plane_wave_block(c64* S, size_t n, int kstride, int col0, int ncol, int nb, const int* q, const c64* pol,
                     hipStream_t s) {
  const unsigned gx = (unsigned)std::min<size_t>((n + 255) / 256, 1024);
  k_plane_waves<<<dim3(gx, ncol, nb), 256, 0, s>>>(S, n, n / 3, kstride, col0, ncol, q, pol);
  KC_LAUNCHED();
  return KC_OK;
}

int random_block(c64* S, size_t n, int kstride, int col0, int ncol, int nb, uint64_t seed, const int* kglobal,
                 hipStream_t s) {
  const unsigned gx = (unsigned)std::max<size_t>(1, std::min<size_t>((n + 255) / 256, 1024));
  dim3 grid(gx, ncol, nb);
  k_random_block<<<grid, 256, 0, s>>>(S, n, kstride, col0, ncol, seed, kglobal);
  KC_LAUNCHED();
  return KC_OK;
}

}  // namespace kc
