// Small dense steps of the LOBPCG iteration, one workgroup (1024 threads) per k-point, all in
// LDS and FP64: masked Cholesky, triangular solves, cyclic Jacobi for complex Hermitian
// matrices with a parallel (round-robin) pair ordering, Ritz-vector selection and the
// construction of the next search direction P orthogonal to the new Ritz vectors.
//
// Columns of S = [X W P] can be inactive (soft-locked bands, dropped directions, or no P yet):
// an inactive column is replaced by the identity in the Gram matrix GB and by an isolated
// diagonal entry above the active spectrum in GA, so it never enters the selected Ritz
// vectors and its coefficients are zero.
#include <algorithm>
#include <cmath>

#include "kc_blas.h"

namespace kc {

// LD: leading dimension of the n x n matrices (RR_NMAX, matrices in LDS; RR_NMAX_WIDE, matrices in
// global memory, for blocks of more than 21 columns per k-point)

// elements per k-point of the Lsave workspace: the saved Cholesky factor, and in the wide form
// (GLOBAL) the working matrices Am, Bm and C1 after it
template <int LD, bool GLOBAL>
constexpr size_t rr_ws_elems() {
  constexpr int LDC = LD == RR_NMAX ? 24 : 32;
  return (size_t)LD * LD + (GLOBAL ? (size_t)2 * LD * LD + (size_t)LD * LDC : 0);
}

// In-place right-looking Cholesky A = L L^H (lower triangle, leading dimension LD) of the
// Hermitian n x n matrix.  A column whose pivot is not above tol * diag0[j] (or is not
// finite) is dropped: its row and column of L become the identity, act[j] = 0, and if it is
// `protect`ed the breakdown flag is raised.  The factor then belongs to the matrix with that
// row and column replaced by the identity.
template <int LD>
__device__ void chol_masked(c64* A, int n, int* act, const double* diag0, double tol, const int* protect,
                            int* breakdown) {
  __shared__ double piv;
  __shared__ int fail;
  __shared__ c64 colj[LD];
  for (int j = 0; j < n; ++j) {
    if (threadIdx.x == 0) {
      const double d = A[j * LD + j].re;
      const bool ok = act[j] && (d > tol * diag0[j]) && std::isfinite(d);
      fail = !ok;
      piv = ok ? sqrt(d) : 1.0;
      if (!ok && act[j]) {
        act[j] = 0;
        if (protect && protect[j]) *breakdown = 1;
      }
    }
    __syncthreads();
    if (fail) {
      for (int t = threadIdx.x; t < n; t += blockDim.x) {
        if (t < j) A[j * LD + t] = mk(0.0, 0.0);
        if (t > j) A[t * LD + j] = mk(0.0, 0.0);
      }
      if (threadIdx.x == 0) A[j * LD + j] = mk(1.0, 0.0);
      __syncthreads();
      continue;
    }
    const double ip = 1.0 / piv;
    for (int t = j + 1 + threadIdx.x; t < n; t += blockDim.x) {
      const c64 v = ip * A[t * LD + j];
      A[t * LD + j] = v;
      colj[t] = v;  // contiguous copy: the update below reads it along k without bank conflicts
    }
    if (threadIdx.x == 0) A[j * LD + j] = mk(piv, 0.0);
    __syncthreads();
    const int m = n - j - 1;
    for (int e = threadIdx.x; e < m * m; e += blockDim.x) {
      const int i = j + 1 + e / m, k = j + 1 + e % m;
      if (k <= i) A[i * LD + k] = A[i * LD + k] - colj[i] * conj(colj[k]);
    }
    __syncthreads();
  }
}

// B <- L^{-1} B for an n x ncol matrix B (leading dimension ldb), L lower (LD).
template <int LD>
__device__ void trsm_lower(const c64* L, int n, c64* B, int ldb, int ncol) {
  for (int c = threadIdx.x; c < ncol; c += blockDim.x) {
    for (int i = 0; i < n; ++i) {
      c64 s = B[i * ldb + c];
      for (int k = 0; k < i; ++k) s = s - L[i * LD + k] * B[k * ldb + c];
      B[i * ldb + c] = (1.0 / L[i * LD + i].re) * s;
    }
  }
  __syncthreads();
}

// B <- L^{-H} B (back substitution with L^H).
template <int LD>
__device__ void trsm_lower_h(const c64* L, int n, c64* B, int ldb, int ncol) {
  for (int c = threadIdx.x; c < ncol; c += blockDim.x) {
    for (int i = n - 1; i >= 0; --i) {
      c64 s = B[i * ldb + c];
      for (int k = i + 1; k < n; ++k) s = s - conj(L[k * LD + i]) * B[k * ldb + c];
      B[i * ldb + c] = (1.0 / L[i * LD + i].re) * s;
    }
  }
  __syncthreads();
}

// in-place conjugate transpose of an n x n LDS matrix (LD)
template <int LD>
__device__ void conj_transpose(c64* A, int n) {
  for (int e = threadIdx.x; e < n * n; e += blockDim.x) {
    const int i = e / n, j = e % n;
    if (i < j) {
      const c64 a = A[i * LD + j], b = A[j * LD + i];
      A[i * LD + j] = conj(b);
      A[j * LD + i] = conj(a);
    } else if (i == j) {
      A[i * LD + i] = mk(A[i * LD + i].re, -A[i * LD + i].im);
    }
  }
  __syncthreads();
}

// Cyclic Jacobi for the Hermitian n x n matrix A (LD) restricted to the active indices (the
// others are isolated: zero rows and columns off the diagonal), accumulating V <- V J.  A
// rotation of the pair (p, q) with a_pq = |a_pq| u, tau = (a_qq - a_pp)/(2|a_pq|),
// t = sign(tau)/(|tau| + sqrt(1 + tau^2)), c = 1/sqrt(1 + t^2), s = t c, uses
// J = [[c, s u], [-s conj(u), c]] on the (p, q) plane and annihilates a_pq.  Pairs come from
// the round-robin schedule (na-1 rounds of na/2 disjoint pairs per sweep over the na active
// indices); one round updates every 2x2 block A[{p_k,q_k},{p_l,q_l}] <- J_k^H A J_l at once.
// Rotations with |a_pq| <= 1e-15 sqrt(|a_pp a_qq|) are skipped; sweeps stop when none is applied.
// A pair is rotated while |a_pq| > 1e-15 sqrt(|a_pp a_qq|) (relative accuracy) and |a_pq| is
// above the rounding floor 4e-16 ||A||_F that the 2x2 updates themselves leave behind; without
// the second test, pairs of a small and a large diagonal entry would keep rotating on noise.
template <int LD>
__device__ void jacobi(c64* A, c64* V, int n, const int* act, double fro) {
  __shared__ int idx[LD];
  __shared__ int na;
  __shared__ int pp[LD / 2], qq[LD / 2];
  __shared__ double cc[LD / 2], ss[LD / 2];
  __shared__ c64 uu[LD / 2];
  __shared__ int nrot;
  if (threadIdx.x == 0) {
    int c = 0;
    for (int i = 0; i < n; ++i)
      if (act[i]) idx[c++] = i;
    na = c;
  }
  __syncthreads();
  const int ne = (na + 1) & ~1;  // even number of players (position na is a dummy when na is odd)
  const int half = ne / 2;
  if (ne < 2) return;
  for (int sweep = 0; sweep < 40; ++sweep) {
    if (threadIdx.x == 0) nrot = 0;
    __syncthreads();
    for (int r = 0; r < ne - 1; ++r) {
      // circle method: position ne-1 fixed, pairs (r, ne-1) and ((r+k) mod (ne-1), (r-k) mod (ne-1))
      for (int k = threadIdx.x; k < half; k += blockDim.x) {
        int a, b;
        if (k == 0) {
          a = r;
          b = ne - 1;
        } else {
          a = (r + k) % (ne - 1);
          b = (r - k + (ne - 1)) % (ne - 1);
        }
        const int lo = min(a, b), hi = max(a, b);
        int p = idx[lo], q = (hi < na) ? idx[hi] : -1;  // q < 0: p is paired with the dummy
        double c = 1.0, s = 0.0;
        c64 u = mk(1.0, 0.0);
        if (q >= 0) {
          const c64 apq = A[p * LD + q];
          const double g = sqrt(abs2(apq));
          const double app = A[p * LD + p].re, aqq = A[q * LD + q].re;
          if (g > 1e-300 && g > 1e-15 * sqrt(fabs(app * aqq)) && g > 4e-16 * fro) {
            const double tau = (aqq - app) / (2.0 * g);
            const double t = (tau >= 0.0 ? 1.0 : -1.0) / (fabs(tau) + sqrt(1.0 + tau * tau));
            c = 1.0 / sqrt(1.0 + t * t);
            s = t * c;
            u = mk(apq.re / g, apq.im / g);
            atomicAdd(&nrot, 1);
          }
        }
        pp[k] = p;
        qq[k] = q;
        cc[k] = c;
        ss[k] = s;
        uu[k] = u;
      }
      __syncthreads();
      // all 2x2 blocks at once: B <- J_k^H B J_l (rows of pair k, columns of pair l)
      for (int e = threadIdx.x; e < half * half; e += blockDim.x) {
        const int k = e / half, l = e % half;
        const int pk = pp[k], qk = qq[k], pl = pp[l], ql = qq[l];
        const double ck = cc[k], sk = ss[k], cl = cc[l], sl = ss[l];
        const c64 uk = uu[k], ul = uu[l];
        c64 b00 = A[pk * LD + pl];
        c64 b01 = (ql >= 0) ? A[pk * LD + ql] : mk(0.0, 0.0);
        c64 b10 = (qk >= 0) ? A[qk * LD + pl] : mk(0.0, 0.0);
        c64 b11 = (qk >= 0 && ql >= 0) ? A[qk * LD + ql] : mk(0.0, 0.0);
        // columns: B J_l
        const c64 c00 = cl * b00 - sl * cmulc(ul, b01), c01 = sl * (ul * b00) + cl * b01;
        const c64 c10 = cl * b10 - sl * cmulc(ul, b11), c11 = sl * (ul * b10) + cl * b11;
        // rows: J_k^H (.)
        c64 d00 = ck * c00 - sk * (uk * c10), d01 = ck * c01 - sk * (uk * c11);
        c64 d10 = sk * cmulc(uk, c00) + ck * c10, d11 = sk * cmulc(uk, c01) + ck * c11;
        if (k == l) {  // the rotated pair: exact zero off the diagonal, real diagonal
          d00 = mk(d00.re, 0.0);
          d11 = mk(d11.re, 0.0);
          d01 = mk(0.0, 0.0);
          d10 = mk(0.0, 0.0);
        }
        A[pk * LD + pl] = d00;
        if (ql >= 0) A[pk * LD + ql] = d01;
        if (qk >= 0) A[qk * LD + pl] = d10;
        if (qk >= 0 && ql >= 0) A[qk * LD + ql] = d11;
      }
      // eigenvectors: V <- V J (all rows); consecutive lanes take different pairs of one row, so
      // their LDS addresses fall in different banks (a column walk would hit one bank)
      for (int e = threadIdx.x; e < half * n; e += blockDim.x) {
        const int i = e / half, l = e % half;
        const int p = pp[l], q = qq[l];
        if (q < 0) continue;
        const double c = cc[l], s = ss[l];
        const c64 u = uu[l];
        const c64 vp = V[i * LD + p], vq = V[i * LD + q];
        V[i * LD + p] = c * vp - s * cmulc(u, vq);
        V[i * LD + q] = s * (u * vp) + c * vq;
      }
      __syncthreads();
    }
    if (nrot == 0) break;
    __syncthreads();
  }
}

// ------------------------------------------------------------------------------------
// Rayleigh-Ritz.  Dynamic LDS: Am (LD x LD), Bm (LD x LD), C1 (LD x mb).
// ------------------------------------------------------------------------------------
template <int LD, bool GLOBAL>
__global__ __launch_bounds__(RR_THREADS) void k_small_rr(const c64* __restrict__ GA, const c64* __restrict__ GB, int mb,
                                                  const int* __restrict__ xmask, const int* __restrict__ wmask,
                                                  const int* __restrict__ pmask, double* __restrict__ theta,
                                                  c64* __restrict__ Cu, int* __restrict__ pvalid,
                                                  c64* __restrict__ Lsave, int* __restrict__ flags,
                                                  const int* __restrict__ kskip, c64* __restrict__ gapp_out,
                                                  const double* __restrict__ res) {
  const int b = blockIdx.x;
  if (kskip && kskip[b]) return;
  constexpr int LDC = LD == RR_NMAX ? 24 : 32;  // leading dim of n x mb blocks (mb <= 21, or 32)
  // this k-point's saved Cholesky factor, then (wide form) its working matrices
  c64* Ls = Lsave + (size_t)b * rr_ws_elems<LD, GLOBAL>();
  extern __shared__ c64 sm[];
  c64* Am = GLOBAL ? Ls + LD * LD : sm;
  c64* Bm = Am + LD * LD;
  c64* C1 = Am + 2 * LD * LD;  // n x mb
  __shared__ int act[LD], prot[LD], ord[LD], pact[LD];
  __shared__ double ev[LD], d0[LD], sc[LD];
  __shared__ int brk, nact;
  __shared__ double fro;
  const int n = 3 * mb;
  const c64* ga = GA + (size_t)b * n * n;
  const c64* gb = GB + (size_t)b * n * n;
  for (int i = threadIdx.x; i < n; i += blockDim.x) {
    act[i] = (i < mb) ? xmask[b * mb + i] : (i < 2 * mb) ? wmask[b * mb + i - mb] : pmask[b * mb + i - 2 * mb];
    prot[i] = (i < mb) ? 1 : 0;
  }
  if (threadIdx.x == 0) {
    brk = 0;
    fro = 0.0;
  }
  __syncthreads();
  // GB, masked and Hermitian
  for (int e = threadIdx.x; e < n * n; e += blockDim.x) {
    const int i = e / n, j = e % n;
    const c64 a = gb[(size_t)i * n + j], c = gb[(size_t)j * n + i];
    c64 h = mk(0.5 * (a.re + c.re), 0.5 * (a.im - c.im));
    if (i == j) h = act[i] ? mk(h.re, 0.0) : mk(1.0, 0.0);
    else if (!act[i] || !act[j]) h = mk(0.0, 0.0);
    Bm[i * LD + j] = h;
  }
  __syncthreads();
  // scale the pencil to unit diagonal (columns of S are not normalised); a zero or non-finite
  // column is dropped (an X column dropping is a breakdown)
  for (int i = threadIdx.x; i < n; i += blockDim.x) {
    const double d = Bm[i * LD + i].re;
    const bool ok = d > 1e-300 && std::isfinite(d);
    if (!ok && act[i] && prot[i]) brk = 1;
    if (!ok) act[i] = 0;
    sc[i] = (ok && act[i]) ? 1.0 / sqrt(d) : 1.0;
    d0[i] = 1.0;
  }
  __syncthreads();
  for (int e = threadIdx.x; e < n * n; e += blockDim.x) {
    const int i = e / n, j = e % n;
    Bm[i * LD + j] = (!act[i] || !act[j]) ? (i == j ? mk(1.0, 0.0) : mk(0.0, 0.0))
                                          : (sc[i] * sc[j]) * Bm[i * LD + j];
  }
  __syncthreads();
  chol_masked<LD>(Bm, n, act, d0, 1e-8, prot, &brk);
  // GA, masked and Hermitian (inactive: zero row/column, diagonal set after the transform)
  for (int e = threadIdx.x; e < n * n; e += blockDim.x) {
    const int i = e / n, j = e % n;
    const c64 a = ga[(size_t)i * n + j], c = ga[(size_t)j * n + i];
    c64 h = mk(0.5 * (a.re + c.re), 0.5 * (a.im - c.im));
    if (i == j) h = mk(h.re, 0.0);
    if (!act[i] || !act[j]) h = mk(0.0, 0.0);
    Am[i * LD + j] = (sc[i] * sc[j]) * h;
  }
  __syncthreads();
  // Am <- L^{-1} Am L^{-H}
  trsm_lower<LD>(Bm, n, Am, LD, n);
  conj_transpose<LD>(Am, n);
  trsm_lower<LD>(Bm, n, Am, LD, n);
  for (int e = threadIdx.x; e < n * n; e += blockDim.x) {
    const int i = e / n, j = e % n;
    if (i < j) {
      const c64 a = Am[i * LD + j], c = Am[j * LD + i];
      const c64 h = mk(0.5 * (a.re + c.re), 0.5 * (a.im - c.im));
      Am[i * LD + j] = h;
      Am[j * LD + i] = conj(h);
    }
  }
  __syncthreads();
  {  // ||A||_F over the active part: per-thread sums, wave sums by shuffles, then the waves
    double f = 0.0;
    for (int e = threadIdx.x; e < n * n; e += blockDim.x) {
      const int i = e / n, j = e % n;
      if (act[i] && act[j]) f += abs2(Am[i * LD + j]);
    }
    for (int o = 32; o > 0; o >>= 1) f += __shfl_down(f, o, 64);
    if ((threadIdx.x & 63) == 0) ev[threadIdx.x >> 6] = f;  // ev is free until the Jacobi ends
    __syncthreads();
    if (threadIdx.x == 0) {
      double t = 0.0;
      for (int w = 0; w < RR_THREADS / 64; ++w) t += ev[w];
      int na = 0;
      for (int i = 0; i < n; ++i) na += act[i] ? 1 : 0;
      fro = sqrt(t);
      nact = na;
      if (!std::isfinite(t) || na < mb) brk = 1;
    }
  }
  __syncthreads();
  for (int i = threadIdx.x; i < n; i += blockDim.x)
    if (!act[i]) Am[i * LD + i] = mk(2.0 * fro + 1.0 + (double)i, 0.0);
  // save L, V = I
  for (int e = threadIdx.x; e < n * n; e += blockDim.x) {
    const int i = e / n, j = e % n;
    Ls[i * LD + j] = Bm[i * LD + j];
    Bm[i * LD + j] = (i == j) ? mk(1.0, 0.0) : mk(0.0, 0.0);
  }
  __syncthreads();
  jacobi<LD>(Am, Bm, n, act, fro);
  // ascending order by rank (ties by index)
  for (int i = threadIdx.x; i < n; i += blockDim.x) ev[i] = Am[i * LD + i].re;
  __syncthreads();
  for (int i = threadIdx.x; i < n; i += blockDim.x) {
    int r = 0;
    for (int j = 0; j < n; ++j) r += (ev[j] < ev[i]) || (ev[j] == ev[i] && j < i);
    ord[r] = i;
  }
  __syncthreads();
  // Plausibility of the new Ritz values.  The search space contains the current X (orthonormal,
  // Ritz values theta_old, residuals R = AX - X Theta), so in exact arithmetic the j-th new Ritz
  // value lies in [lambda_j, theta_old_j] (Cauchy interlacing: it cannot rise) and
  // lambda_j >= theta_old_j - |R|_2 (the eigenvalues
  // of A are within |R|_2 of those of Theta), |R|_2 <= (sum_j |r_j|^2)^(1/2), when X holds the
  // lowest eigenvectors' neighbourhood; the operator is
  // positive semi-definite as well.  A value below both bounds can only come from a pencil that
  // lost its rank in rounding (seen when the residuals sit at the rounding floor of the FP64
  // application): with a complete X block the step is then rejected -- X and its image stay, P
  // is dropped, and the host restarts the iteration from X (flag 2).
  __shared__ int reject;
  if (threadIdx.x == 0) {
    bool xfull = true;
    for (int i = 0; i < mb; ++i) xfull = xfull && act[i];
    reject = 0;
    if (xfull) {
      double r2 = 0.0;
      for (int j = 0; j < mb; ++j) r2 += res ? res[b * mb + j] * res[b * mb + j] : 0.0;
      const double rn = sqrt(r2);
      double tmax = 0.0;
      for (int j = 0; j < mb; ++j) tmax = fmax(tmax, fabs(theta[b * mb + j]));
      // the residual bound is applied only once the block is nearly converged (|R| below 1e-4 of
      // the Ritz values): earlier, a lower eigenvalue that X has not met yet may still enter
      const bool late = res && std::isfinite(rn) && rn < 1e-4 * tmax;
      for (int j = 0; j < mb; ++j) {
        const double t_old = theta[b * mb + j], t_new = ev[ord[j]];
        // below the bound, or above theta_old_j (the Ritz values of a space that contains X do not
        // rise), each with the residual's slack
        const double slack = 2.0 * rn + 1e-10 * fabs(t_old);
        if (t_new < -1e-8 * fro || (late && (t_new < t_old - slack || t_new > t_old + slack))) reject = 1;
      }
    }
  }
  __syncthreads();
  if (reject) {
    for (int j = threadIdx.x; j < mb; j += blockDim.x) {
      const double gbj = gb[(size_t)j * n + j].re;
      theta[b * mb + j] = gbj > 0.0 ? ga[(size_t)j * n + j].re / gbj : 0.0;
      pvalid[b * mb + j] = 0;
    }
    c64* out = Cu + (size_t)b * n * 2 * mb;
    for (int e = threadIdx.x; e < n * 2 * mb; e += blockDim.x) {
      const int i = e / (2 * mb), j = e % (2 * mb);
      out[e] = (j < mb && i == j) ? mk(1.0, 0.0) : mk(0.0, 0.0);
    }
    if (gapp_out)
      for (int e = threadIdx.x; e < mb * mb; e += blockDim.x) gapp_out[(size_t)b * mb * mb + e] = mk(0.0, 0.0);
    if (threadIdx.x == 0) atomicOr(&flags[b], 2);
    return;
  }
  for (int j = threadIdx.x; j < mb; j += blockDim.x) theta[b * mb + j] = ev[ord[j]];
  // C1 = L^{-H} V[:, ord[0..mb)]
  for (int e = threadIdx.x; e < n * mb; e += blockDim.x) {
    const int i = e / mb, j = e % mb;
    C1[i * LDC + j] = Bm[i * LD + ord[j]];
  }
  for (int e = threadIdx.x; e < n * n; e += blockDim.x) {
    const int i = e / n, j = e % n;
    Am[i * LD + j] = Ls[i * LD + j];
  }
  __syncthreads();
  trsm_lower_h<LD>(Am, n, C1, LDC, mb);
  // P direction: Y = C1 with the X rows zeroed; Y' = Y - C1 (C1^H GB Y); Y'' = Y' M^{-1/2}
  // through the Cholesky factor of M = Y'^H GB Y'.  Bm <- GB (masked), Am regions:
  c64* GY = Am;                    // n x mb (LDC)
  c64* T = Am + LD * LDC;          // mb x mb (LDC)
  c64* Yp = T + LDC * LDC;         // n x mb (LDC); ends below LD*LD
  for (int e = threadIdx.x; e < n * n; e += blockDim.x) {
    const int i = e / n, j = e % n;
    const c64 a = gb[(size_t)i * n + j], c = gb[(size_t)j * n + i];
    c64 h = mk(0.5 * (a.re + c.re), 0.5 * (a.im - c.im));
    if (i == j) h = act[i] ? mk(h.re, 0.0) : mk(1.0, 0.0);
    else if (!act[i] || !act[j]) h = mk(0.0, 0.0);
    Bm[i * LD + j] = (act[i] && act[j]) ? (sc[i] * sc[j]) * h : h;
  }
  __syncthreads();
  for (int e = threadIdx.x; e < n * mb; e += blockDim.x) {  // GY = GB Y
    const int i = e / mb, j = e % mb;
    c64 s = mk(0.0, 0.0);
    for (int k = mb; k < n; ++k) s = s + Bm[i * LD + k] * C1[k * LDC + j];
    GY[i * LDC + j] = s;
  }
  __syncthreads();
  for (int e = threadIdx.x; e < mb * mb; e += blockDim.x) {  // T = C1^H GY
    const int i = e / mb, j = e % mb;
    c64 s = mk(0.0, 0.0);
    for (int k = 0; k < n; ++k) s = s + cmulc(C1[k * LDC + i], GY[k * LDC + j]);
    T[i * LDC + j] = s;
  }
  __syncthreads();
  for (int e = threadIdx.x; e < n * mb; e += blockDim.x) {  // Y' = Y - C1 T
    const int i = e / mb, j = e % mb;
    c64 s = (i >= mb) ? C1[i * LDC + j] : mk(0.0, 0.0);
    for (int k = 0; k < mb; ++k) s = s - C1[i * LDC + k] * T[k * LDC + j];
    Yp[i * LDC + j] = s;
  }
  __syncthreads();
  for (int e = threadIdx.x; e < n * mb; e += blockDim.x) {  // GY = GB Y'
    const int i = e / mb, j = e % mb;
    c64 s = mk(0.0, 0.0);
    for (int k = 0; k < n; ++k) s = s + Bm[i * LD + k] * Yp[k * LDC + j];
    GY[i * LDC + j] = s;
  }
  __syncthreads();
  // M = Y'^H GB Y' into Bm (mb x mb, LD), then Cholesky with drops
  for (int e = threadIdx.x; e < mb * mb; e += blockDim.x) {
    const int i = e / mb, j = e % mb;
    c64 s = mk(0.0, 0.0);
    for (int k = 0; k < n; ++k) s = s + cmulc(Yp[k * LDC + i], GY[k * LDC + j]);
    Bm[i * LD + j] = s;
  }
  __syncthreads();
  for (int e = threadIdx.x; e < mb * mb; e += blockDim.x) {
    const int i = e / mb, j = e % mb;
    if (i < j) {
      const c64 a = Bm[i * LD + j], c = Bm[j * LD + i];
      const c64 h = mk(0.5 * (a.re + c.re), 0.5 * (a.im - c.im));
      Bm[i * LD + j] = h;
      Bm[j * LD + i] = conj(h);
    } else if (i == j) {
      Bm[i * LD + i] = mk(Bm[i * LD + i].re, 0.0);
    }
  }
  // scale M to unit diagonal (the P candidates of nearly converged bands are tiny but still
  // carry a direction); a zero or non-finite column is dropped
  for (int i = threadIdx.x; i < mb; i += blockDim.x) {
    const double d = Bm[i * LD + i].re;
    const bool ok = d > 1e-300 && std::isfinite(d);
    pact[i] = ok ? 1 : 0;
    ev[i] = ok ? 1.0 / sqrt(d) : 0.0;  // column scales
    d0[i] = 1.0;
  }
  __syncthreads();
  for (int e = threadIdx.x; e < mb * mb; e += blockDim.x) {
    const int i = e / mb, j = e % mb;
    Bm[i * LD + j] = (ev[i] * ev[j]) * Bm[i * LD + j];
  }
  for (int e = threadIdx.x; e < n * mb; e += blockDim.x) {
    const int i = e / mb, j = e % mb;
    Yp[i * LDC + j] = ev[j] * Yp[i * LDC + j];
  }
  __syncthreads();
  chol_masked<LD>(Bm, mb, pact, d0, 1e-10, nullptr, &brk);
  // Y''^H = L_M^{-1} Y'^H (mb x n, leading dim LD) over the dead GY/T regions (below Yp)
  c64* YH = Am;
  __syncthreads();
  for (int e = threadIdx.x; e < mb * n; e += blockDim.x) {
    const int i = e / n, c = e % n;
    YH[i * LD + c] = conj(Yp[c * LDC + i]);
  }
  __syncthreads();
  trsm_lower<LD>(Bm, mb, YH, LD, n);
  c64* out = Cu + (size_t)b * n * 2 * mb;
  for (int e = threadIdx.x; e < n * 2 * mb; e += blockDim.x) {
    const int i = e / (2 * mb), j = e % (2 * mb);
    c64 v;
    if (j < mb) v = C1[i * LDC + j];
    else v = pact[j - mb] ? conj(YH[(j - mb) * LD + i]) : mk(0.0, 0.0);
    out[e] = sc[i] * v;  // back to the unscaled columns of S
  }
  for (int j = threadIdx.x; j < mb; j += blockDim.x) pvalid[b * mb + j] = pact[j];
  if (threadIdx.x == 0 && brk) atomicOr(&flags[b], 1);
  if (gapp_out) {
    // P_new^H A P_new = Cp^H GA Cp over the active columns, for the next step's Gram blocks
    __syncthreads();
    c64* T1 = Bm;  // n x mb (LDC)
    auto cup = [&](int i, int a) -> c64 { return pact[a] ? sc[i] * conj(YH[a * LD + i]) : mk(0.0, 0.0); };
    for (int e = threadIdx.x; e < n * mb; e += blockDim.x) {
      const int i = e / mb, a = e % mb;
      c64 acc = mk(0.0, 0.0);
      if (act[i])
        for (int j = 0; j < n; ++j)
          if (act[j]) {
            const c64 x = ga[(size_t)i * n + j], y = ga[(size_t)j * n + i];
            acc = acc + mk(0.5 * (x.re + y.re), 0.5 * (x.im - y.im)) * cup(j, a);
          }
      T1[i * LDC + a] = acc;
    }
    __syncthreads();
    for (int e = threadIdx.x; e < mb * mb; e += blockDim.x) {
      const int a = e / mb, c = e % mb;
      c64 acc = mk(0.0, 0.0);
      for (int i = 0; i < n; ++i)
        if (act[i]) acc = acc + cmulc(cup(i, a), T1[i * LDC + c]);
      gapp_out[((size_t)b * mb + a) * mb + c] = acc;
    }
  }
}

int small_rr(const c64* GA, const c64* GB, int mb, int nb, const int* xmask, const int* wmask, const int* pmask,
             double* theta, c64* Cu, int* pvalid, c64* Lsave, int* flags, const int* kskip, c64* gapp_out,
             hipStream_t s, const double* res) {
  if (3 * mb > RR_NMAX_WIDE || mb > 32) {
    set_error("block size too large");
    return KC_ERR_INVALID_ARG;
  }
  if (3 * mb > RR_NMAX || mb > 21) {
    // wide blocks: the matrices do not fit in LDS and live in the Lsave workspace (L2-resident)
    k_small_rr<RR_NMAX_WIDE, true><<<nb, RR_THREADS, 0, s>>>(GA, GB, mb, xmask, wmask, pmask, theta, Cu, pvalid, Lsave,
                                                             flags, kskip, gapp_out, res);
    KC_LAUNCHED();
    return KC_OK;
  }
  constexpr int LD = RR_NMAX;
  const size_t shm = (size_t)(2 * LD * LD + LD * 24) * sizeof(c64);
  static bool attr = false;
  if (!attr) {
    KC_HIP(hipFuncSetAttribute((const void*)k_small_rr<RR_NMAX, false>, hipFuncAttributeMaxDynamicSharedMemorySize,
                               (int)shm));
    attr = true;
  }
  k_small_rr<RR_NMAX, false><<<nb, RR_THREADS, shm, s>>>(GA, GB, mb, xmask, wmask, pmask, theta, Cu, pvalid, Lsave,
                                                         flags, kskip, gapp_out, res);
  KC_LAUNCHED();
  return KC_OK;
}

size_t small_rr_ws_bytes(int mb) {
  const bool wide = 3 * mb > RR_NMAX || mb > 21;
  return (wide ? rr_ws_elems<RR_NMAX_WIDE, true>() : rr_ws_elems<RR_NMAX, false>()) * sizeof(c64);
}

}  // namespace kc
