// Launchers of the LOBPCG block kernels (kc_blas.hip) and small dense kernels (kc_small.hip).
#pragma once

#include "kc_state.h"

namespace kc {

// GA_b = S_b^H AS_b, GB_b = S_b^H S_b (nc x nc, complex, row-major [nb][nc][nc]); columns of
// k-point b start at (b * kstride) * n.  `part` is scratch.
int gram2(const c64* S, const c64* AS, int kstride, int nc, size_t n, int nb, DevBuf& part, c64* GA, c64* GB,
          const int* kskip, hipStream_t s);
// The same with caller-provided partial sums (gram2_part_bytes(nc, n, nb) bytes).
int gram2(const c64* S, const c64* AS, int kstride, int nc, size_t n, int nb, c64* part, c64* GA, c64* GB,
          const int* kskip, hipStream_t s);
size_t gram2_part_bytes(int nc, size_t n, int nb);
// gram2 (contiguous blocks, kstride = nc) with its partial sums in a buffer of part_bytes bytes:
// the chunks are made longer (fewer partial sums) until they fit; KC_ERR_INVALID_ARG when even
// one chunk per k-point does not.
int gram2_bounded(const c64* S, const c64* AS, int nc, size_t n, int nb, c64* part, size_t part_bytes, c64* GA,
                  c64* GB, hipStream_t s);

// The W columns of the Gram matrices of S = [X W P] (kstride-spaced blocks of 3mb columns):
// GB(:, W) = S^H W, GA(:, W) = S^H AW, with the X/P blocks filled from the previous
// Rayleigh-Ritz step: GB_XX = GB_PP = I, GB_XP = 0, GA_XX = diag(theta), GA_XP = 0,
// GA_PP = gapp ([nb][mb][mb]).  Valid while X and P are the last Rayleigh-Ritz output and AX, AP
// their updated images.
int gramw(const c64* S, const c64* AS, int kstride, int mb, size_t n, int nb, DevBuf& part, c64* GA, c64* GB,
          const double* theta, const c64* gapp, const int* kskip, hipStream_t s);

// Y_b[:, map(j)] = S_b[:, scol0 .. scol0+p) C_b, C: [nb][p][q]; output column j < q goes to
// ycol0 + j (j < q1) or ycol1 + j - q1; Y may alias S.
int update(const c64* S, int skstride, int scol0, int p, c64* Y, int ykstride, int q, int q1, int ycol0,
           int ycol1, const c64* C, size_t n, int nb, const int* kskip, hipStream_t s);

// Workgroups per k-point of update and update_res (update_res's partial sums take
// nb * mb * update_grid_x(n, nb) * 2 doubles).
unsigned update_grid_x(size_t n, int nb);

// Both updates of a Rayleigh-Ritz step and the next residuals in one pass (S, AS: kstride-spaced
// groups of 3mb columns [X W P], C: [nb][3mb][2mb]): [X P] <- S C, [AX AP] <- AS C in place,
// R_j = AX_j - theta_j X_j into R ([nb*mb][n]), res_j = |r_j| / |x_j| and xnorm2_j = |x_j|^2.
int update_res(c64* S, c64* AS, int kstride, int mb, const c64* C, size_t n, int nb, const double* theta, c64* R,
               double* part, double* res, double* xnorm2, const int* kskip, hipStream_t s);
// Sets the LDS limit of update_res's kernels (call once before update_res is captured in a graph).
int update_res_prepare();

// W_j = K_P^{-1} (AX_j - theta_j X_j), res_j = |AX_j - theta_j X_j| / |X_j|; optionally the
// residuals themselves (Rout, contiguous [nb*mb][3N^3]) and |r_j|^2 (rnorm2); W is left
// untouched for the k-points b with wskip[b] != 0.  sfl (device double [nb], or nullptr): per
// k-point floor of s = |K|^2 in the gains 1/s and 1/(gamma s) (the frequency s = 0 stays zero).
int resid_precond(const c64* S, const c64* AS, c64* W, const double* theta, const c64* ktab64,
                  const double* gamma, int N, int kstride, int xcol0, int wcol0, int mb, int nb, DevBuf& part,
                  double* res, double* xnorm2, const int* kskip, hipStream_t s, c64* Rout = nullptr,
                  double* rnorm2 = nullptr, const int* wskip = nullptr, const double* sfl = nullptr,
                  const Skew* sk = nullptr);

// Removes the DC longitudinal direction (x(0) along conj(K(0))) from columns [col0, col0 + ncol)
// of the k-points b with dcl[b] != 0 (kstride-spaced groups; FP64).
int deflate_dc_long(c64* S, int kstride, int col0, int ncol, int nb, const c64* ktab64, int N, const int* dcl,
                    hipStream_t s);

int random_block(c64* S, size_t n, int kstride, int col0, int ncol, int nb, uint64_t seed, const int* kglobal,
                 hipStream_t s);
// columns [col0, col0 + ncol) of each k-point's group: the plane waves q (device int [nb][ncol],
// flattened frequency; q < 0 leaves the column) with polarizations pol (device c64 [nb][ncol][3])
int plane_wave_block(c64* S, size_t n, int kstride, int col0, int ncol, int nb, const int* q, const c64* pol,
                     hipStream_t s);

// Small dense steps (one workgroup per k-point), see kc_small.hip.
constexpr int RR_NMAX = 64;       // 3 * block size of the LDS-resident kernels (block size <= 21)
constexpr int RR_NMAX_WIDE = 96;  // 3 * block size of the wide path (block size <= 32)
constexpr int RR_THREADS = 1024;  // one workgroup per k-point: 16 waves hide the LDS latency

// Rayleigh-Ritz on S = [X W P]: from GA = S^H AS, GB = S^H S (3mb x 3mb) compute the mb
// smallest Ritz values theta and Cu = [C1 | Cp] (3mb x 2mb) with X_new = S C1, P_new = S Cp
// (P_new orthonormal and orthogonal to X_new in the GB inner product).  The columns of S need
// not be normalised or orthogonal: the pencil is scaled to unit diagonal first.
// Also writes gapp_out[b] = P_new^H A P_new = Cp^H GA Cp (mb x mb) for the next step's gramw.
// res (device [nb * mb], or nullptr): the current residual norms |r_j| of the (orthonormal) X
// block, theta its current Ritz values: a step whose Ritz values fall below what they allow is
// rejected (X kept, P dropped, flags[b] |= 2).
// Blocks of up to 21 columns (3mb <= RR_NMAX) keep the matrices in LDS; wider ones (mb <= 32) in
// Lsave, which holds small_rr_ws_bytes(mb) bytes per k-point.
int small_rr(const c64* GA, const c64* GB, int mb, int nb, const int* xmask, const int* wmask, const int* pmask,
             double* theta, c64* Cu, int* pvalid, c64* Lsave, int* flags, const int* kskip, c64* gapp_out,
             hipStream_t s, const double* res = nullptr);
size_t small_rr_ws_bytes(int mb);

}  // namespace kc
