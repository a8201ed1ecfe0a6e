// Matrix-free application of the kernel-compensated operator in k-space (Prop 2.8,
// eq (2.30)) and of the diagonal-block preconditioner (eqs (2.31)-(2.32)) on gfx950.
//
// y = K_A F3^H M F3 K_A^H x + gamma K_B x is evaluated in pencil passes over the
// [vec][3][z][y][x] layout, each pass one round trip of the block through HBM:
//
//   X1  e = -conj(K) x x (curl symbol, prologue), inverse DFT along x         (3 comps);
//       also K . x per point for the penalty term of X2
//   Y1  inverse DFT along y                                                   (per comp)
//   Z   Trivial/diagonal: inverse DFT along z, E' = M E / N^3 pointwise,
//       forward DFT along z                                                   (3 comps)
//       CrossDoF: Za inverse DFT along z (per comp); Zb E' = M E / N^3 with the
//       four-point cross-DoF averages read around each point, forward DFT along z
//   Y2  forward DFT along y                                                   (per comp)
//   X2  forward DFT along x, y = K x e' + gamma conj(K) (K . x) (epilogue)
//
// The 1D symbols K_a(q) = (1 - e^{-i theta_q})/h + i k_a (1 + e^{-i theta_q})/2 are read from
// a table of 3N entries per k-point (eq (2.28)), so no per-frequency array is stored.
//
// The same passes evaluate the transverse-projection preconditioner
//   T_E r = K_A^{+H} F3^H E F3 K_A^{+} r + (gamma K_B)^{+} r,
// the pseudo-inverse of Op with the inverse permittivity replaced by a positive diagonal
// field E (the permittivity itself, in the classical choice E_c = 1/(eps^-1)_cc at the
// c-edge points).  Each symbol factors as K_a = i e^{-i theta_a/2} kappa_a with kappa_a
// real, so K_A = [K x] is a unitary rescaling of the real cross-product matrix [kappa x] and
// K_A^{+} = K_A^H / s with s = |K_1|^2 + |K_2|^2 + |K_3|^2; likewise (gamma K_B)^{+} =
// K_B / (gamma s^2).  Hence T_E r = (1/s) [K_A F3^H E F3 K_A^H (r/s) + (1/gamma) K_B (r/s)]:
// the operator's passes with a 1/s prologue and epilogue, the diagonal field E in the Z pass
// and 1/gamma for gamma.  T_E is Hermitian positive semi-definite, zero exactly where K_P is
// singular, and equals K_P^{-1} for E = 1.  The field scales each component separately, so in
// FP32 with the field shared by all k-points the y and z work of T_E is one pass over whole
// yz-planes in LDS (k_yz_field), between x-passes that write and read an x-major layout.
#include <algorithm>
#include <cmath>
#include <type_traits>
#include <vector>

#include "kc_fft.h"
#include "kc_state.h"

namespace kc {

constexpr int NT = 256;

template <int N, int NC, typename T>
struct TileP {
  static constexpr int P0 = (NC == 3 && sizeof(T) == 8 && N >= 64) ? 8 : 16;
  static constexpr int P = (N % P0 == 0) ? P0
                           : (N % 8 == 0) ? 8
                           : (N % 4 == 0) ? 4
                           : (N % 2 == 0) ? 2
                                          : 1;
};

template <typename T>
__device__ __forceinline__ void load_eps_table(EpsEntry<T>* lt, const EpsEntry<T>* gt, int n_mat) {
  for (int t = threadIdx.x; t < n_mat; t += blockDim.x) lt[t] = gt[t];
}

// ------------------------------------------------------------------------------------
// X1: curl prologue + inverse DFT along x.  Tile: P rows (y) of one (vec, z), 3 comps.  With XT
// the output is written x-major, [vec][c][x][z][y], for the yz-plane pass (P consecutive y of
// one (x, z) are contiguous there).
// ------------------------------------------------------------------------------------
template <int N, typename T, bool PRE, int P, bool XT = false>
__global__ __launch_bounds__(NT) void k_x1_curl_inv(const c64* __restrict__ x, cpx<T>* __restrict__ E,
                                                    const cpx<T>* __restrict__ ktab, VecMap vm,
                                                    const cpx<T>* __restrict__ gtw, cpx<T>* __restrict__ kx,
                                                    const c64* __restrict__ ktab64, c64* __restrict__ kx64,
                                                    const double* __restrict__ sfl, Skew sk) {
  using G = TileGeom<N, P, 3>;
  __shared__ cpx<T> lds[G::ELEMS];
  __shared__ cpx<T> tw[N];
  constexpr size_t N3 = (size_t)N * N * N;
  // x-major: the tiles yt, yt + 1 share 128-byte lines, so they go to the same XCD (one L2)
  unsigned b = XT ? xcd_swizzle(blockIdx.x, gridDim.x) : blockIdx.x;
  const int yt = b % (N / P);
  b /= (N / P);
  const int z = b % N;
  const int vec = b / N;
  if (!vm.on(vec)) return;
  const cpx<T>* K = ktab + (size_t)(vec / vm.vpk) * 3 * N;
  load_twiddles<N>(tw, gtw);
  const c64* xv = x + vm.off(vec) * 3 * N3;
  for (int w = threadIdx.x; w < N * P; w += NT) {
    const int e = w % N, p = w / N, y = yt * P + p;
    const size_t off = (size_t)z * N * N + (size_t)y * N + e;
    const cpx<T> x1 = cvt<T>(xv[off]), x2 = cvt<T>(xv[N3 + off]), x3 = cvt<T>(xv[2 * N3 + off]);
    cpx<T> K1 = K[e], K2 = K[N + y], K3 = K[2 * N + z];
    skew_fix<T>(sk, e, y, z, K1, K2, K3);
    const cpx<T> v1 = conj(K1), v2 = conj(K2), v3 = conj(K3);
    cpx<T> c1 = v3 * x2 - v2 * x3, c2 = v1 * x3 - v3 * x1, c3 = v2 * x1 - v1 * x2;
    // the penalty term of the last pass needs only K . x: kept here (FP64 for the operator,
    // the compute precision for the preconditioner), so that pass does not re-read x
    if constexpr (PRE && XT) kx[(size_t)vec * N3 + off] = cmulc(v1, x1) + cmulc(v2, x2) + cmulc(v3, x3);
    if constexpr (!PRE) {
      const c64* Kd = ktab64 + (size_t)(vec / vm.vpk) * 3 * N;
      c64 K1d = Kd[e], K2d = Kd[N + y], K3d = Kd[2 * N + z];
      skew_fix<double>(sk, e, y, z, K1d, K2d, K3d);
      kx64[(size_t)vec * N3 + off] = K1d * xv[off] + K2d * xv[N3 + off] + K3d * xv[2 * N3 + off];
    }
    if (PRE) {  // K_A^{+} = K_A^H / s (s floored at sfl near k = 0)
      const T sq = abs2(v1) + abs2(v2) + abs2(v3);
      const T fl = sfl ? static_cast<T>(sfl[vec / vm.vpk]) : T(0);
      const T is = sq > T(0) ? T(1) / (sq < fl ? fl : sq) : T(0);
      c1 = is * c1;
      c2 = is * c2;
      c3 = is * c3;
    }
    lds[G::addr3(0, e, p)] = c1;
    lds[G::addr3(1, e, p)] = c2;
    lds[G::addr3(2, e, p)] = c3;
  }
  __syncthreads();
  fft_tile<N, P, 3, NT, +1, T>(lds, tw);
  cpx<T>* Ev = E + (size_t)vec * 3 * N3;
  if constexpr (XT) {
    for (int w = threadIdx.x; w < 3 * N * P; w += NT) {
      const int p = w % P, e = (w / P) % N, c = w / (N * P);
      Ev[c * N3 + (size_t)e * N * N + (size_t)z * N + yt * P + p] = lds[G::addr3(c, e, p)];
    }
  } else {
    for (int w = threadIdx.x; w < 3 * N * P; w += NT) {
      const int e = w % N, p = (w / N) % P, c = w / (N * P), y = yt * P + p;
      Ev[c * N3 + (size_t)z * N * N + (size_t)y * N + e] = lds[G::addr3(c, e, p)];
    }
  }
}

// ------------------------------------------------------------------------------------
// X2: forward DFT along x + outer curl + penalty epilogue (XT: input x-major, as X1 writes it).
// ------------------------------------------------------------------------------------
template <int N, typename T, bool PRE, int P, bool XT = false>
__global__ __launch_bounds__(NT) void k_x2_fwd_curl_pen(const cpx<T>* __restrict__ E,
                                                        const c64* __restrict__ x, c64* __restrict__ y,
                                                        const cpx<T>* __restrict__ ktab,
                                                        const c64* __restrict__ ktab64,
                                                        const double* __restrict__ gamma,
                                                        VecMap vm, VecMap vmy, const cpx<T>* __restrict__ gtw,
                                                        const cpx<T>* __restrict__ kxin, const c64* __restrict__ kx64,
                                                        const double* __restrict__ sfl, Skew sk) {
  using G = TileGeom<N, P, 3>;
  __shared__ cpx<T> lds[G::ELEMS];
  __shared__ cpx<T> tw[N];
  constexpr size_t N3 = (size_t)N * N * N;
  // x-major: the tiles yt, yt + 1 share 128-byte lines, so they go to the same XCD (one L2)
  unsigned b = XT ? xcd_swizzle(blockIdx.x, gridDim.x) : blockIdx.x;
  const int yt = b % (N / P);
  b /= (N / P);
  const int z = b % N;
  const int vec = b / N;
  if (!vm.on(vec)) return;
  const int ik = vec / vm.vpk;
  const cpx<T>* K = ktab + (size_t)ik * 3 * N;
  const c64* Kd = ktab64 + (size_t)ik * 3 * N;
  const double g = PRE ? 1.0 / gamma[ik] : gamma[ik];
  load_twiddles<N>(tw, gtw);
  const cpx<T>* Ev = E + (size_t)vec * 3 * N3;
  if constexpr (XT) {
    for (int w = threadIdx.x; w < 3 * N * P; w += NT) {
      const int p = w % P, e = (w / P) % N, c = w / (N * P);
      lds[G::addr3(c, e, p)] = Ev[c * N3 + (size_t)e * N * N + (size_t)z * N + yt * P + p];
    }
  } else {
    for (int w = threadIdx.x; w < 3 * N * P; w += NT) {
      const int e = w % N, p = (w / N) % P, c = w / (N * P), yy = yt * P + p;
      lds[G::addr3(c, e, p)] = Ev[c * N3 + (size_t)z * N * N + (size_t)yy * N + e];
    }
  }
  __syncthreads();
  fft_tile<N, P, 3, NT, -1, T>(lds, tw);
  const c64* xv = x + vm.off(vec) * 3 * N3;
  c64* yv = y + vmy.off(vec) * 3 * N3;
  for (int w = threadIdx.x; w < N * P; w += NT) {
    const int e = w % N, p = w / N, yy = yt * P + p;
    const size_t off = (size_t)z * N * N + (size_t)yy * N + e;
    const cpx<T> e1 = lds[G::addr3(0, e, p)], e2 = lds[G::addr3(1, e, p)], e3 = lds[G::addr3(2, e, p)];
    cpx<T> K1 = K[e], K2 = K[N + yy], K3 = K[2 * N + z];
    skew_fix<T>(sk, e, yy, z, K1, K2, K3);
    const c64 c1 = cvt<double>(K2 * e3 - K3 * e2);
    const c64 c2 = cvt<double>(K3 * e1 - K1 * e3);
    const c64 c3 = cvt<double>(K1 * e2 - K2 * e1);
    c64 K1d = Kd[e], K2d = Kd[N + yy], K3d = Kd[2 * N + z];
    skew_fix<double>(sk, e, yy, z, K1d, K2d, K3d);
    c64 kx;  // K . x
    if constexpr (PRE && XT) {
      kx = cvt<double>(kxin[(size_t)vec * N3 + off]);
    } else if constexpr (!PRE) {
      kx = kx64[(size_t)vec * N3 + off];
    } else {
      const c64 x1 = xv[off], x2 = xv[N3 + off], x3 = xv[2 * N3 + off];
      kx = K1d * x1 + K2d * x2 + K3d * x3;
    }
    if (PRE) {  // (1/s) [c + (1/gamma) K_B x / s], the outer 1/s floored at sfl near k = 0
      const double sq = abs2(K1d) + abs2(K2d) + abs2(K3d);
      const double fl = sfl ? sfl[ik] : 0.0;
      const double is = sq > 0.0 ? 1.0 / sq : 0.0, ie = sq < fl ? 1.0 / fl : is;
      const c64 gk = (g * is) * kx;
      yv[off] = ie * (c1 + cmulc(K1d, gk));
      yv[N3 + off] = ie * (c2 + cmulc(K2d, gk));
      yv[2 * N3 + off] = ie * (c3 + cmulc(K3d, gk));
    } else {
      const c64 gk = g * kx;
      yv[off] = c1 + cmulc(K1d, gk);
      yv[N3 + off] = c2 + cmulc(K2d, gk);
      yv[2 * N3 + off] = c3 + cmulc(K3d, gk);
    }
  }
}

// ------------------------------------------------------------------------------------
// Y: DFT along y, in place.  Tile: P consecutive x of one (vec*3+c, z).
// ------------------------------------------------------------------------------------
template <int N, int DIR, typename T, int P>
__global__ __launch_bounds__(NT) void k_y(cpx<T>* __restrict__ buf, const cpx<T>* __restrict__ gtw,
                                          const int* __restrict__ active) {
  using G = TileGeom<N, P, 1>;
  __shared__ cpx<T> lds[G::ELEMS];
  __shared__ cpx<T> tw[N];
  constexpr size_t N3 = (size_t)N * N * N;
  unsigned b = blockIdx.x;
  const int xt = b % (N / P);
  b /= (N / P);
  const int z = b % N;
  const size_t vc = b / N;
  if (active && !active[vc / 3]) return;
  load_twiddles<N>(tw, gtw);
  cpx<T>* base = buf + vc * N3 + (size_t)z * N * N + xt * P;
  for (int w = threadIdx.x; w < N * P; w += NT) {
    const int p = w % P, e = w / P;
    lds[G::addr3(0, e, p)] = base[(size_t)e * N + p];
  }
  __syncthreads();
  fft_tile<N, P, 1, NT, DIR, T>(lds, tw);
  for (int w = threadIdx.x; w < N * P; w += NT) {
    const int p = w % P, e = w / P;
    base[(size_t)e * N + p] = lds[G::addr3(0, e, p)];
  }
}

// ------------------------------------------------------------------------------------
// X (plain): DFT along x, in -> out (out may alias in).  Tile: P rows of one (vc, z).
// ------------------------------------------------------------------------------------
template <int N, int DIR, typename T, int P>
__global__ __launch_bounds__(NT) void k_x_plain(const cpx<T>* in, cpx<T>* out, const cpx<T>* __restrict__ gtw) {
  using G = TileGeom<N, P, 1>;
  __shared__ cpx<T> lds[G::ELEMS];
  __shared__ cpx<T> tw[N];
  constexpr size_t N3 = (size_t)N * N * N;
  unsigned b = blockIdx.x;
  const int yt = b % (N / P);
  b /= (N / P);
  const int z = b % N;
  const size_t vc = b / N;
  load_twiddles<N>(tw, gtw);
  const size_t base = vc * N3 + (size_t)z * N * N + (size_t)yt * P * N;
  for (int w = threadIdx.x; w < N * P; w += NT) {
    const int e = w % N, p = w / N;
    lds[G::addr3(0, e, p)] = in[base + (size_t)p * N + e];
  }
  __syncthreads();
  fft_tile<N, P, 1, NT, DIR, T>(lds, tw);
  for (int w = threadIdx.x; w < N * P; w += NT) {
    const int e = w % N, p = w / N;
    out[base + (size_t)p * N + e] = lds[G::addr3(0, e, p)];
  }
}

// ------------------------------------------------------------------------------------
// Z (plain): DFT along z, in -> out (may alias).  Tile: P consecutive x of one (vc, y).
// ------------------------------------------------------------------------------------
template <int N, int DIR, typename T, int P>
__global__ __launch_bounds__(NT) void k_z_plain(const cpx<T>* in, cpx<T>* out, const cpx<T>* __restrict__ gtw,
                                                const int* __restrict__ active, int ncomp) {
  using G = TileGeom<N, P, 1>;
  __shared__ cpx<T> lds[G::ELEMS];
  __shared__ cpx<T> tw[N];
  constexpr size_t N3 = (size_t)N * N * N;
  unsigned b = blockIdx.x;
  const int xt = b % (N / P);
  b /= (N / P);
  const int yy = b % N;
  const size_t vc = b / N;
  if (active && !active[vc / ncomp]) return;
  load_twiddles<N>(tw, gtw);
  const size_t base = vc * N3 + (size_t)yy * N + xt * P;
  for (int w = threadIdx.x; w < N * P; w += NT) {
    const int p = w % P, e = w / P;
    lds[G::addr3(0, e, p)] = in[base + (size_t)e * N * N + p];
  }
  __syncthreads();
  fft_tile<N, P, 1, NT, DIR, T>(lds, tw);
  for (int w = threadIdx.x; w < N * P; w += NT) {
    const int p = w % P, e = w / P;
    out[base + (size_t)e * N * N + p] = lds[G::addr3(0, e, p)];
  }
}

// ------------------------------------------------------------------------------------
// Z (Trivial / diagonal): inverse DFT along z, pointwise 3x3 Hermitian inverse permittivity
// (diagonal from the edge points, off-diagonals from the volume point; eqs (3.3)-(3.4)),
// forward DFT along z.  In place.  Tile: P consecutive x of one (vec, y), 3 comps.
// ------------------------------------------------------------------------------------
template <int N, typename T, int P>
__global__ __launch_bounds__(NT) void k_z_trivial(cpx<T>* __restrict__ buf, const uint32_t* __restrict__ ids,
                                                  const EpsEntry<T>* __restrict__ geps, int n_mat,
                                                  const cpx<T>* __restrict__ gtw, const int* __restrict__ active) {
  using G = TileGeom<N, P, 3>;
  __shared__ cpx<T> lds[G::ELEMS];
  __shared__ cpx<T> tw[N];
  __shared__ EpsEntry<T> eps[KC_MAX_MAT];
  constexpr size_t N3 = (size_t)N * N * N;
  unsigned b = blockIdx.x;
  const int xt = b % (N / P);
  b /= (N / P);
  const int yy = b % N;
  const size_t vec = b / N;
  if (active && !active[vec]) return;
  load_twiddles<N>(tw, gtw);
  load_eps_table(eps, geps, n_mat);
  cpx<T>* base = buf + vec * 3 * N3 + (size_t)yy * N + xt * P;
  for (int w = threadIdx.x; w < 3 * N * P; w += NT) {
    const int p = w % P, e = (w / P) % N, c = w / (N * P);
    lds[G::addr3(c, e, p)] = base[c * N3 + (size_t)e * N * N + p];
  }
  __syncthreads();
  fft_tile<N, P, 3, NT, +1, T>(lds, tw);
  for (int w = threadIdx.x; w < N * P; w += NT) {
    const int p = w % P, e = w / P;
    const uint32_t id = ids[(size_t)e * N * N + (size_t)yy * N + xt * P + p];
    const EpsEntry<T>& ax = eps[id & 255u];
    const EpsEntry<T>& ay = eps[(id >> 8) & 255u];
    const EpsEntry<T>& az = eps[(id >> 16) & 255u];
    const EpsEntry<T>& av = eps[id >> 24];
    const cpx<T> E1 = lds[G::addr3(0, e, p)], E2 = lds[G::addr3(1, e, p)], E3 = lds[G::addr3(2, e, p)];
    const cpx<T> o12 = av.o[0], o13 = av.o[1], o23 = av.o[2];
    lds[G::addr3(0, e, p)] = ax.d[0] * E1 + o12 * E2 + o13 * E3;
    lds[G::addr3(1, e, p)] = cmulc(o12, E1) + ay.d[1] * E2 + o23 * E3;
    lds[G::addr3(2, e, p)] = cmulc(o13, E1) + cmulc(o23, E2) + az.d[2] * E3;
  }
  __syncthreads();
  fft_tile<N, P, 3, NT, -1, T>(lds, tw);
  for (int w = threadIdx.x; w < 3 * N * P; w += NT) {
    const int p = w % P, e = (w / P) % N, c = w / (N * P);
    base[c * N3 + (size_t)e * N * N + p] = lds[G::addr3(c, e, p)];
  }
}

// ------------------------------------------------------------------------------------
// Z (transverse-projection preconditioner): inverse DFT along z, E_c' = f_c E_c / N^3 with a
// positive per-point field f (FP32 [3][N^3], one per k-point group or shared), forward DFT
// along z.  In place.  Tile: P consecutive x of one (vec, y), 3 comps.
// ------------------------------------------------------------------------------------
template <int N, typename T, int P>
__global__ __launch_bounds__(NT) void k_z_field(cpx<T>* __restrict__ buf, const float* __restrict__ field,
                                                int vpk, int fkstride, const cpx<T>* __restrict__ gtw,
                                                const int* __restrict__ active) {
  using G = TileGeom<N, P, 3>;
  __shared__ cpx<T> lds[G::ELEMS];
  __shared__ cpx<T> tw[N];
  constexpr size_t N3 = (size_t)N * N * N;
  constexpr T inv = T(1) / T(N3);
  unsigned b = blockIdx.x;
  const int xt = b % (N / P);
  b /= (N / P);
  const int yy = b % N;
  const size_t vec = b / N;
  if (active && !active[vec]) return;
  load_twiddles<N>(tw, gtw);
  const float* f = field + (size_t)(vec / vpk) * fkstride * 3 * N3;
  cpx<T>* base = buf + vec * 3 * N3 + (size_t)yy * N + xt * P;
  for (int w = threadIdx.x; w < 3 * N * P; w += NT) {
    const int p = w % P, e = (w / P) % N, c = w / (N * P);
    lds[G::addr3(c, e, p)] = base[c * N3 + (size_t)e * N * N + p];
  }
  __syncthreads();
  fft_tile<N, P, 3, NT, +1, T>(lds, tw);
  for (int w = threadIdx.x; w < 3 * N * P; w += NT) {
    const int p = w % P, e = (w / P) % N, c = w / (N * P);
    const T fc = (T)f[c * N3 + (size_t)e * N * N + (size_t)yy * N + xt * P + p] * inv;
    lds[G::addr3(c, e, p)] = fc * lds[G::addr3(c, e, p)];
  }
  __syncthreads();
  fft_tile<N, P, 3, NT, -1, T>(lds, tw);
  for (int w = threadIdx.x; w < 3 * N * P; w += NT) {
    const int p = w % P, e = (w / P) % N, c = w / (N * P);
    base[c * N3 + (size_t)e * N * N + p] = lds[G::addr3(c, e, p)];
  }
}

// ------------------------------------------------------------------------------------
// YZ (transverse-projection preconditioner, FP32, shared field): on the x-major layout one
// workgroup holds the whole yz-plane of one (vec, component, x) in LDS (N x (N+1) complex, the
// odd pitch spreads the row-wise stages over the banks) and does what the Y1, Z(field) and Y2
// passes do in three round trips: inverse DFTs along y and z, E_c' = f_c E_c / N^3 with the
// x-major field, forward DFTs along z and y.  In place.
// ------------------------------------------------------------------------------------
constexpr int NT_PLANE = 1024;

template <int N, typename T>
constexpr size_t plane_lds_bytes() {
  return ((size_t)N * (N + 1) + N) * sizeof(cpx<T>);
}

// the plane pass is used where its tile fits the 160 KiB of LDS (FP32 up to N = 128)
template <int N, typename T>
constexpr bool plane_ok() {
  return sizeof(T) == 4 && plane_lds_bytes<N, T>() <= 160 * 1024;
}

// Persistent: workgroup b takes the planes b, b + gridDim.x, ... (planes of inactive vectors
// skipped) and loads the next plane into registers while it transforms the current one in LDS
// (the loads stay in flight across the LDS barriers), since a 128 x 128 plane leaves room for
// one workgroup per CU and nothing else would overlap its memory traffic.  The next plane's
// field is loaded after the current one has been multiplied (one register set for it).
template <int N, typename T>
__global__ __launch_bounds__(NT_PLANE) void k_yz_field(cpx<T>* __restrict__ buf, const float* __restrict__ fieldt,
                                                       const cpx<T>* __restrict__ gtw,
                                                       const int* __restrict__ active, int vpk, int fks,
                                                       unsigned nplanes) {
  constexpr int PL = N + 1;
  constexpr size_t N3 = (size_t)N * N * N;
  constexpr T inv = T(1) / T(N3);
  constexpr int PER = (N * N + NT_PLANE - 1) / NT_PLANE;  // plane entries per thread
  extern __shared__ __align__(16) unsigned char plane_smem[];
  cpx<T>* lds = reinterpret_cast<cpx<T>*>(plane_smem);
  cpx<T>* tw = lds + N * PL;
  load_twiddles<N>(tw, gtw);  // visible after the first barrier below
  // plane p: x = p % N of component c = (p / N) % 3 of vector p / 3N, [z][y]
  auto next_from = [&](unsigned p) {
    while (p < nplanes && active && !active[p / (3 * N)]) p += gridDim.x;
    return p;
  };
  auto plane = [&](unsigned p) { return buf + (size_t)p * N * N; };
  auto field = [&](unsigned p) {
    const size_t vec = p / (3 * N);
    return fieldt + (size_t)(vec / vpk) * fks * 3 * N3 + (size_t)(p % (3 * N)) * N * N;
  };
  cpx<T> nv[PER];
  float nf[PER];
  auto load_plane_regs = [&](unsigned p) {
    const cpx<T>* pl = plane(p);
#pragma unroll
    for (int i = 0; i < PER; ++i) {
      const int t = threadIdx.x + i * NT_PLANE;
      if ((N * N) % NT_PLANE == 0 || t < N * N) nv[i] = pl[t];
    }
  };
  auto load_field_regs = [&](unsigned p) {
    const float* f = field(p);
#pragma unroll
    for (int i = 0; i < PER; ++i) {
      const int t = threadIdx.x + i * NT_PLANE;
      if ((N * N) % NT_PLANE == 0 || t < N * N) nf[i] = f[t];
    }
  };
  unsigned p = next_from(blockIdx.x);
  if (p < nplanes) {
    load_plane_regs(p);
    load_field_regs(p);
  }
  while (p < nplanes) {
    const unsigned pn = next_from(p + gridDim.x);
    __syncthreads();  // the previous plane's last LDS reads are done
#pragma unroll
    for (int i = 0; i < PER; ++i) {
      const int t = threadIdx.x + i * NT_PLANE;
      if ((N * N) % NT_PLANE == 0 || t < N * N) lds[(t / N) * PL + t % N] = nv[i];
    }
    if (pn < nplanes) load_plane_regs(pn);
    __syncthreads();
    fft_2d<N, N, 1, PL, NT_PLANE, +1, T>(lds, tw);  // along y: pencils = rows z
    fft_2d<N, N, PL, 1, NT_PLANE, +1, T>(lds, tw);  // along z: pencils = columns y
#pragma unroll
    for (int i = 0; i < PER; ++i) {
      const int t = threadIdx.x + i * NT_PLANE;
      if ((N * N) % NT_PLANE == 0 || t < N * N) {
        const int a = (t / N) * PL + t % N;
        lds[a] = ((T)nf[i] * inv) * lds[a];
      }
    }
    if (pn < nplanes) load_field_regs(pn);
    __syncthreads();
    fft_2d<N, N, PL, 1, NT_PLANE, -1, T>(lds, tw);
    fft_2d<N, N, 1, PL, NT_PLANE, -1, T>(lds, tw);
    cpx<T>* pl = plane(p);
    for (int t = threadIdx.x; t < N * N; t += NT_PLANE) pl[t] = lds[(t / N) * PL + t % N];
    p = pn;
  }
}

// ------------------------------------------------------------------------------------
// Zb (CrossDoF): E' = M_CrossDoF E / N^3 (eq (3.8)) evaluated around each point from the
// real-space field E, then forward DFT along z.  With Q^(e)_cd the (c,d) entry of the
// inverse permittivity at the e-edge points and T_cd the four-point averages of eq (3.7),
// block (c,d), c < d, is (Q^(c)_cd T_cd + T_cd Q^(d)_cd)/2, so at a point P
//   [block(c,d) E_d](P) = 1/8 sum_{S in T_cd-stencil(P)} (Q^(c)_cd(P) + Q^(d)_cd(S)) E_d(S)
// and the lower blocks are the conjugate transposes.  Stencils (0-based, periodic):
//   T12: (i,j),(i-1,j),(i,j+1),(i-1,j+1)   T13: (i,k),(i-1,k),(i,k+1),(i-1,k+1)
//   T23: (j,k),(j-1,k),(j,k+1),(j-1,k+1)   and their transposes mirrored.
// Tile: P consecutive x of one (vec, y), 3 comps.  A thread walks a segment of z for one x: the
// stencils need E1 at the columns (i,j), (i+1,j), (i,j-1), (i+1,j-1), E2 at (i,j), (i-1,j),
// (i,j+1), (i-1,j+1), E3 at (i,j), (i-1,j), (i,j-1), and the ids at those seven columns, on the
// planes k-1, k, k+1; the three planes live in registers and slide along z, so each plane is
// read once per thread.  E and ids are read through the cache (neighbouring tiles share them).
// Where no material couples z to x or y ((eps^-1)_13 = (eps^-1)_23 = 0, e.g. gyrotropic media
// magnetised along z) the blocks (1,3), (2,3) and their transposes are zero and the kernel
// (ZOFF = false) reads and multiplies only the in-plane stencils of plane k.
// ------------------------------------------------------------------------------------
template <typename T>
struct ZPlane {
  cpx<T> e1[4];    // E1 at (i,j), (i+1,j), (i,j-1), (i+1,j-1)
  cpx<T> e2[4];    // E2 at (i,j), (i-1,j), (i,j+1), (i-1,j+1)
  cpx<T> e3[3];    // E3 at (i,j), (i-1,j), (i,j-1)
  uint32_t id[7];  // ids at (i,j), (i+1,j), (i,j-1), (i+1,j-1), (i-1,j), (i,j+1), (i-1,j+1)
};

// 32-bit byte offsets from a uniform base: the loads take the scalar-base + vector-offset form
template <typename T>
__device__ __forceinline__ T ld_off(const T* base, uint32_t byte_off) {
  return *reinterpret_cast<const T*>(reinterpret_cast<const char*>(base) + byte_off);
}

// ZOFF == false: only the values of the in-plane blocks (1,2), (2,1) and the diagonal
template <bool ZOFF = true, typename T>
__device__ __forceinline__ void load_plane(ZPlane<T>& z, const cpx<T>* E1, const cpx<T>* E2, const cpx<T>* E3,
                                           const uint32_t* ids, const uint32_t (&col)[7], uint32_t plane) {
  // col: (i,j), (i+1,j), (i,j-1), (i+1,j-1), (i-1,j), (i,j+1), (i-1,j+1)
  uint32_t o[7];
#pragma unroll
  for (int c = 0; c < 7; ++c) o[c] = plane + col[c];
  constexpr uint32_t B = sizeof(cpx<T>);
  z.e1[0] = ld_off(E1, o[0] * B);
  z.e1[1] = ld_off(E1, o[1] * B);
  z.e1[2] = ld_off(E1, o[2] * B);
  z.e1[3] = ld_off(E1, o[3] * B);
  z.e2[0] = ld_off(E2, o[0] * B);
  z.e2[1] = ld_off(E2, o[4] * B);
  z.e2[2] = ld_off(E2, o[5] * B);
  z.e2[3] = ld_off(E2, o[6] * B);
  z.e3[0] = ld_off(E3, o[0] * B);
  if constexpr (ZOFF) {
    z.e3[1] = ld_off(E3, o[4] * B);
    z.e3[2] = ld_off(E3, o[2] * B);
  }
#pragma unroll
  for (int c = 0; c < 7; ++c) z.id[c] = ld_off(ids, o[c] * 4u);
}

template <int N, int P>
struct ZbSeg {  // z-segments per x: the largest divisor of N with P * NSEG <= 256 threads
  static constexpr int pick() {
    int best = 1;
    for (int d = 1; d <= N; ++d)
      if (N % d == 0 && P * d <= 256) best = d;
    return best;
  }
  static constexpr int NSEG = pick();
  static constexpr int ZL = N / NSEG;
};

template <int N, typename T, int P, bool ZOFF>
__global__ __launch_bounds__(NT) void k_zb_crossdof(const cpx<T>* __restrict__ E, cpx<T>* __restrict__ out,
                                                    const uint32_t* __restrict__ ids,
                                                    const EpsEntry<T>* __restrict__ geps, int n_mat,
                                                    const cpx<T>* __restrict__ gtw, const int* __restrict__ active) {
  using G = TileGeom<N, P, 3>;
  constexpr int NSEG = ZbSeg<N, P>::NSEG, ZL = ZbSeg<N, P>::ZL;
  __shared__ cpx<T> lds[G::ELEMS];
  __shared__ cpx<T> tw[N];
  // the permittivity table, n_mat entries (dynamic LDS: the tile and this table fit three
  // workgroups per CU at N = 128, P = 16 in FP32)
  extern __shared__ __align__(16) unsigned char zb_eps_smem[];
  EpsEntry<T>* eps = reinterpret_cast<EpsEntry<T>*>(zb_eps_smem);
  constexpr size_t N3 = (size_t)N * N * N;
  constexpr uint32_t NN = (uint32_t)N * N;
  const unsigned nb = gridDim.x;
  unsigned b = xcd_swizzle(blockIdx.x, nb);
  const int xt = b % (N / P);
  b /= (N / P);
  const int yy = b % N;
  const size_t vec = b / N;
  if (active && !active[vec]) return;
  load_twiddles<N>(tw, gtw);
  load_eps_table(eps, geps, n_mat);
  __syncthreads();
  const cpx<T>* E1 = E + vec * 3 * N3;
  const cpx<T>* E2 = E1 + N3;
  const cpx<T>* E3 = E2 + N3;
  const T e8 = static_cast<T>(0.125);
  for (int w = threadIdx.x; w < P * NSEG; w += NT) {
    const int p = w % P, seg = w / P;
    const int i = xt * P + p, j = yy;
    const int ip = (i + 1 == N) ? 0 : i + 1, im = (i == 0) ? N - 1 : i - 1;
    const int jp = (j + 1 == N) ? 0 : j + 1, jm = (j == 0) ? N - 1 : j - 1;
    const uint32_t col[7] = {(uint32_t)(j * N + i),  (uint32_t)(j * N + ip), (uint32_t)(jm * N + i),
                             (uint32_t)(jm * N + ip), (uint32_t)(j * N + im), (uint32_t)(jp * N + i),
                             (uint32_t)(jp * N + im)};
    const int kb = seg * ZL;
    if constexpr (!ZOFF) {
      // (eps^-1)_13 = (eps^-1)_23 = 0 in every material: the blocks (1,3), (2,3) and their
      // transposes vanish, and each plane needs only its own values
#pragma unroll
      for (int t = 0; t < ZL; ++t) {
        const int k = kb + t;
        ZPlane<T> cur;
        load_plane<false>(cur, E1, E2, E3, ids, col, (uint32_t)k * NN);
        const uint32_t idc = cur.id[0];
        const EpsEntry<T>& ex = eps[idc & 255u];
        const EpsEntry<T>& ey = eps[(idc >> 8) & 255u];
        const EpsEntry<T>& ez = eps[(idc >> 16) & 255u];
        auto mx = [&](uint32_t id) -> const EpsEntry<T>& { return eps[id & 255u]; };
        auto my = [&](uint32_t id) -> const EpsEntry<T>& { return eps[(id >> 8) & 255u]; };
        cpx<T> a1 = mk(T(0), T(0));
        cfma(a1, ex.o[0] + my(cur.id[0]).o[0], cur.e2[0]);
        cfma(a1, ex.o[0] + my(cur.id[4]).o[0], cur.e2[1]);
        cfma(a1, ex.o[0] + my(cur.id[5]).o[0], cur.e2[2]);
        cfma(a1, ex.o[0] + my(cur.id[6]).o[0], cur.e2[3]);
        cpx<T> a2 = mk(T(0), T(0));
        cfmac(a2, mx(cur.id[0]).o[0] + ey.o[0], cur.e1[0]);
        cfmac(a2, mx(cur.id[1]).o[0] + ey.o[0], cur.e1[1]);
        cfmac(a2, mx(cur.id[2]).o[0] + ey.o[0], cur.e1[2]);
        cfmac(a2, mx(cur.id[3]).o[0] + ey.o[0], cur.e1[3]);
        lds[G::addr3(0, k, p)] = ex.d[0] * cur.e1[0] + e8 * a1;
        lds[G::addr3(1, k, p)] = ey.d[1] * cur.e2[0] + e8 * a2;
        lds[G::addr3(2, k, p)] = ez.d[2] * cur.e3[0];
      }
      continue;
    }
    ZPlane<T> prev, cur, next;
    load_plane(prev, E1, E2, E3, ids, col, (uint32_t)(kb == 0 ? N - 1 : kb - 1) * NN);
    load_plane(cur, E1, E2, E3, ids, col, (uint32_t)kb * NN);
    // fully unrolled (ZL is a compile-time constant): the three planes rotate by renaming, not
    // by register moves
#pragma unroll
    for (int t = 0; t < ZL; ++t) {
      const int k = kb + t;
      load_plane(next, E1, E2, E3, ids, col, (uint32_t)(k + 1 == N ? 0 : k + 1) * NN);
      const uint32_t idc = cur.id[0];
      const EpsEntry<T>& ex = eps[idc & 255u];
      const EpsEntry<T>& ey = eps[(idc >> 8) & 255u];
      const EpsEntry<T>& ez = eps[(idc >> 16) & 255u];
      auto mx = [&](uint32_t id) -> const EpsEntry<T>& { return eps[id & 255u]; };
      auto my = [&](uint32_t id) -> const EpsEntry<T>& { return eps[(id >> 8) & 255u]; };
      auto mz = [&](uint32_t id) -> const EpsEntry<T>& { return eps[(id >> 16) & 255u]; };
      // row 1: d1 E1 + block(1,2) E2 [T12 on plane k] + block(1,3) E3 [T13 on planes k, k+1]
      cpx<T> a1 = mk(T(0), T(0));
      cfma(a1, ex.o[0] + my(cur.id[0]).o[0], cur.e2[0]);
      cfma(a1, ex.o[0] + my(cur.id[4]).o[0], cur.e2[1]);
      cfma(a1, ex.o[0] + my(cur.id[5]).o[0], cur.e2[2]);
      cfma(a1, ex.o[0] + my(cur.id[6]).o[0], cur.e2[3]);
      cfma(a1, ex.o[1] + mz(cur.id[0]).o[1], cur.e3[0]);
      cfma(a1, ex.o[1] + mz(cur.id[4]).o[1], cur.e3[1]);
      cfma(a1, ex.o[1] + mz(next.id[0]).o[1], next.e3[0]);
      cfma(a1, ex.o[1] + mz(next.id[4]).o[1], next.e3[1]);
      // row 2: block(2,1) E1 [T21 on plane k] + d2 E2 + block(2,3) E3 [T23 on planes k, k+1]
      cpx<T> a2 = mk(T(0), T(0));
      cfmac(a2, mx(cur.id[0]).o[0] + ey.o[0], cur.e1[0]);
      cfmac(a2, mx(cur.id[1]).o[0] + ey.o[0], cur.e1[1]);
      cfmac(a2, mx(cur.id[2]).o[0] + ey.o[0], cur.e1[2]);
      cfmac(a2, mx(cur.id[3]).o[0] + ey.o[0], cur.e1[3]);
      cfma(a2, ey.o[2] + mz(cur.id[0]).o[2], cur.e3[0]);
      cfma(a2, ey.o[2] + mz(cur.id[2]).o[2], cur.e3[2]);
      cfma(a2, ey.o[2] + mz(next.id[0]).o[2], next.e3[0]);
      cfma(a2, ey.o[2] + mz(next.id[2]).o[2], next.e3[2]);
      // row 3: block(3,1) E1 [T31 on planes k, k-1] + block(3,2) E2 [T32 on planes k, k-1] + d3 E3
      cpx<T> a3 = mk(T(0), T(0));
      cfmac(a3, mx(cur.id[0]).o[1] + ez.o[1], cur.e1[0]);
      cfmac(a3, mx(cur.id[1]).o[1] + ez.o[1], cur.e1[1]);
      cfmac(a3, mx(prev.id[0]).o[1] + ez.o[1], prev.e1[0]);
      cfmac(a3, mx(prev.id[1]).o[1] + ez.o[1], prev.e1[1]);
      cfmac(a3, my(cur.id[0]).o[2] + ez.o[2], cur.e2[0]);
      cfmac(a3, my(cur.id[5]).o[2] + ez.o[2], cur.e2[2]);
      cfmac(a3, my(prev.id[0]).o[2] + ez.o[2], prev.e2[0]);
      cfmac(a3, my(prev.id[5]).o[2] + ez.o[2], prev.e2[2]);
      lds[G::addr3(0, k, p)] = ex.d[0] * cur.e1[0] + e8 * a1;
      lds[G::addr3(1, k, p)] = ey.d[1] * cur.e2[0] + e8 * a2;
      lds[G::addr3(2, k, p)] = ez.d[2] * cur.e3[0] + e8 * a3;
      prev = cur;
      cur = next;
    }
  }
  __syncthreads();
  fft_tile<N, P, 3, NT, -1, T>(lds, tw);
  cpx<T>* base = out + vec * 3 * N3 + (size_t)yy * N + xt * P;
  for (int w = threadIdx.x; w < 3 * N * P; w += NT) {
    const int p = w % P, e = (w / P) % N, c = w / (N * P);
    base[c * N3 + (size_t)e * N * N + p] = lds[G::addr3(c, e, p)];
  }
}

// ------------------------------------------------------------------------------------
// Preconditioner: z = K_P^{-1} r per frequency.  With v = conj(K), s = |K|^2 and
// K_P = s I + (gamma - 1) v v^H (eq (2.31) with K_A K_A^H + K_B = s I, Lemma 2.4 (1)),
// Sherman-Morrison gives K_P^{-1} r = (r - v (v^H r)/s)/s + v (v^H r)/(gamma s^2).
// ------------------------------------------------------------------------------------
__global__ __launch_bounds__(NT) void k_precond(const c64* r, c64* z, const c64* __restrict__ ktab64, Skew sk,
                                                const double* __restrict__ gamma, int N, int nvec,
                                                int vecs_per_k) {
  const size_t N3 = (size_t)N * N * N;
  const size_t tot = N3 * nvec;
  for (size_t t = (size_t)blockIdx.x * NT + threadIdx.x; t < tot; t += (size_t)gridDim.x * NT) {
    const size_t vec = t / N3, p = t - vec * N3;
    const int ik = (int)(vec / vecs_per_k);
    const c64* K = ktab64 + (size_t)ik * 3 * N;
    const int qx = (int)(p % N), qy = (int)((p / N) % N), qz = (int)(p / ((size_t)N * N));
    c64 K1 = K[qx], K2 = K[N + qy], K3 = K[2 * N + qz];
    skew_fix<double>(sk, qx, qy, qz, K1, K2, K3);
    const c64* rv = r + vec * 3 * N3;
    c64* zv = z + vec * 3 * N3;
    const c64 r1 = rv[p], r2 = rv[N3 + p], r3 = rv[2 * N3 + p];
    const double s = abs2(K1) + abs2(K2) + abs2(K3);
    if (s == 0.0) {
      zv[p] = mk(0.0, 0.0);
      zv[N3 + p] = mk(0.0, 0.0);
      zv[2 * N3 + p] = mk(0.0, 0.0);
      continue;
    }
    const double g = gamma[ik];
    const c64 vr = K1 * r1 + K2 * r2 + K3 * r3;  // v^H r with v = conj(K)
    const double is = 1.0 / s;
    const double cf = (1.0 / g - 1.0) * is * is;  // coefficient of v (v^H r)
    const c64 u = cf * vr;
    zv[p] = is * r1 + cmulc(K1, u);
    zv[N3 + p] = is * r2 + cmulc(K2, u);
    zv[2 * N3 + p] = is * r3 + cmulc(K3, u);
  }
}

// ------------------------------------------------------------------------------------
// host launchers
// ------------------------------------------------------------------------------------
static inline unsigned nblk(size_t n) { return (unsigned)n; }

// ------------------------------------------------------------------------------------
// Tile widths.  Every pass handles P pencils per workgroup; any P that divides N and whose
// LDS tile (NC components x N x (P+1) complex, plus twiddles and the permittivity table) fits
// the 64 KiB of static LDS is valid, and the data layout between passes does not depend on it.
// The width of each pass is chosen per handle and precision by timing the candidates
// (tune_tiles); until then, and for grids below 32, TileP's heuristic is used.
// ------------------------------------------------------------------------------------
template <int N, int NC, typename T, int P>
constexpr bool tile_ok() {
  return P >= 1 && N % P == 0 &&
         (size_t)TileGeom<N, P, NC>::ELEMS * sizeof(cpx<T>) + N * sizeof(cpx<T>) + KC_MAX_MAT * sizeof(EpsEntry<T>) <=
             65536;
}

// calls f(std::integral_constant<int, P>) with the requested width if valid, else the default
template <int N, int NC, typename T, typename F>
static void with_tile(int p, F&& f) {
  constexpr int PD = TileP<N, NC, T>::P;
  if (p == 4) {
    if constexpr (tile_ok<N, NC, T, 4>()) return f(std::integral_constant<int, 4>{});
  } else if (p == 8) {
    if constexpr (tile_ok<N, NC, T, 8>()) return f(std::integral_constant<int, 8>{});
  } else if (p == 16) {
    if constexpr (tile_ok<N, NC, T, 16>()) return f(std::integral_constant<int, 16>{});
  } else if (p == 32) {
    if constexpr (tile_ok<N, NC, T, 32>()) return f(std::integral_constant<int, 32>{});
  }
  f(std::integral_constant<int, PD>{});
}

template <int N, int NC, typename T>
static std::vector<int> tile_candidates() {
  std::vector<int> c{TileP<N, NC, T>::P};
  auto add = [&](int p, bool ok) {
    if (ok && std::find(c.begin(), c.end(), p) == c.end()) c.push_back(p);
  };
  if (N >= 32) {
    add(4, tile_ok<N, NC, T, 4>());
    add(8, tile_ok<N, NC, T, 8>());
    add(16, tile_ok<N, NC, T, 16>());
    add(32, tile_ok<N, NC, T, 32>());
  }
  return c;
}

template <typename T>
static int tile_of(const kc_op* op, int pass) {
  return op->tiles[sizeof(T) == 8 ? 1 : 0][pass];
}

// The launchers below take the tile width of their pass from the handle.
template <int N, typename T, bool PRE, bool XT = false>
static void launch_x1(kc_op* op, int pass, int nvec, const c64* x, cpx<T>* A, const cpx<T>* ktab, const VecMap& vm,
                      const cpx<T>* tw, hipStream_t s, cpx<T>* kx = nullptr, const c64* ktab64 = nullptr,
                      c64* kx64 = nullptr, const double* sfl = nullptr) {
  with_tile<N, 3, T>(tile_of<T>(op, pass), [&](auto pc) {
    constexpr int P = decltype(pc)::value;
    k_x1_curl_inv<N, T, PRE, P, XT>
        <<<nblk((size_t)nvec * N * (N / P)), NT, 0, s>>>(x, A, ktab, vm, tw, kx, ktab64, kx64, sfl, op->skew);
  });
}

template <int N, typename T, bool PRE, bool XT = false>
static void launch_x2(kc_op* op, int pass, int nvec, const cpx<T>* A, const c64* x, c64* y, const cpx<T>* ktab,
                      const c64* ktab64, const double* gam, const VecMap& vm, const VecMap& vmy, const cpx<T>* tw,
                      hipStream_t s, const cpx<T>* kx = nullptr, const c64* kx64 = nullptr,
                      const double* sfl = nullptr) {
  with_tile<N, 3, T>(tile_of<T>(op, pass), [&](auto pc) {
    constexpr int P = decltype(pc)::value;
    k_x2_fwd_curl_pen<N, T, PRE, P, XT><<<nblk((size_t)nvec * N * (N / P)), NT, 0, s>>>(
        A, x, y, ktab, ktab64, gam, vm, vmy, tw, kx, kx64, sfl, op->skew);
  });
}

template <int N, typename T>
static void launch_yz(int nvec, cpx<T>* A, const float* fieldt, int vpk, int fks, const cpx<T>* tw, const int* act,
                      hipStream_t s) {
  if constexpr (plane_ok<N, T>()) {
    // one persistent workgroup per plane slot: CUs x the workgroups of 1024 threads that fit (LDS)
    const unsigned np = (unsigned)nvec * 3 * N;
    const unsigned per_cu = plane_lds_bytes<N, T>() > 80 * 1024 ? 1 : 2;
    const unsigned g = std::min<unsigned>(np, 256 * per_cu);
    k_yz_field<N, T><<<g, NT_PLANE, plane_lds_bytes<N, T>(), s>>>(A, fieldt, tw, act, vpk, fks, np);
  }
}

template <int N, int DIR, typename T>
static void launch_y(kc_op* op, int pass, int nvec, cpx<T>* A, const cpx<T>* tw, const int* act, hipStream_t s) {
  with_tile<N, 1, T>(tile_of<T>(op, pass), [&](auto pc) {
    constexpr int P = decltype(pc)::value;
    k_y<N, DIR, T, P><<<nblk((size_t)nvec * 3 * N * (N / P)), NT, 0, s>>>(A, tw, act);
  });
}

template <int N, int DIR, typename T>
static void launch_zplain(kc_op* op, int pass, int nvc, const cpx<T>* in, cpx<T>* out, const cpx<T>* tw,
                          const int* act, int ncomp, hipStream_t s) {
  with_tile<N, 1, T>(tile_of<T>(op, pass), [&](auto pc) {
    constexpr int P = decltype(pc)::value;
    k_z_plain<N, DIR, T, P><<<nblk((size_t)nvc * N * (N / P)), NT, 0, s>>>(in, out, tw, act, ncomp);
  });
}

template <int N, typename T>
static void launch_zb(kc_op* op, int nvec, const cpx<T>* B, cpx<T>* A, const EpsEntry<T>* eps, const cpx<T>* tw,
                      const int* act, hipStream_t s) {
  with_tile<N, 3, T>(tile_of<T>(op, TP_ZB), [&](auto pc) {
    constexpr int P = decltype(pc)::value;
    const size_t lds = op->n_mat * sizeof(EpsEntry<T>);
    const unsigned g = nblk((size_t)nvec * N * (N / P));
    if (op->zoff)
      k_zb_crossdof<N, T, P, true><<<g, NT, lds, s>>>(B, A, op->ids.as<uint32_t>(), eps, op->n_mat, tw, act);
    else
      k_zb_crossdof<N, T, P, false><<<g, NT, lds, s>>>(B, A, op->ids.as<uint32_t>(), eps, op->n_mat, tw, act);
  });
}

template <int N, typename T>
static void launch_zt(kc_op* op, int nvec, cpx<T>* A, const EpsEntry<T>* eps, const cpx<T>* tw, const int* act,
                      hipStream_t s) {
  with_tile<N, 3, T>(tile_of<T>(op, TP_ZT), [&](auto pc) {
    constexpr int P = decltype(pc)::value;
    k_z_trivial<N, T, P><<<nblk((size_t)nvec * N * (N / P)), NT, 0, s>>>(A, op->ids.as<uint32_t>(), eps, op->n_mat,
                                                                         tw, act);
  });
}

template <int N, typename T>
static void launch_zf(kc_op* op, int nvec, cpx<T>* A, const float* field, int vpk, int fks, const cpx<T>* tw,
                      const int* act, hipStream_t s) {
  with_tile<N, 3, T>(tile_of<T>(op, TP_ZF), [&](auto pc) {
    constexpr int P = decltype(pc)::value;
    k_z_field<N, T, P><<<nblk((size_t)nvec * N * (N / P)), NT, 0, s>>>(A, field, vpk, fks, tw, act);
  });
}

template <typename T>
struct PassArgs {
  const cpx<T>* ktab;
  const c64* ktab64;
  const double* gam;
  const cpx<T>* tw;
  const EpsEntry<T>* eps;
};

template <int N, typename T>
static PassArgs<T> pass_args(kc_op* op, int ik0) {
  const bool f64 = sizeof(T) == 8;
  PassArgs<T> a;
  a.ktab = (f64 ? op->ktab64.as<cpx<T>>() : op->ktab32.as<cpx<T>>()) + (size_t)ik0 * 3 * N;
  a.ktab64 = op->ktab64.as<c64>() + (size_t)ik0 * 3 * N;
  a.gam = op->gamma_d.as<double>() + ik0;
  a.tw = f64 ? op->tw64.as<cpx<T>>() : op->tw32.as<cpx<T>>();
  a.eps = f64 ? op->eps64.as<EpsEntry<T>>() : op->eps32.as<EpsEntry<T>>();
  return a;
}

template <int N, typename T>
static int tune_tiles_n(kc_op* op, int nvec, hipStream_t s);

template <int N, typename T>
static int apply_n(kc_op* op, int ik0, int nvec, const VecMap& vm, const c64* x, c64* y, hipStream_t s,
                   hipEvent_t* ev) {
  KC_TRY((tune_tiles_n<N, T>(op, nvec, s)));
  int nev = 0;
  auto mark = [&]() -> int {
    if (ev) KC_HIP(hipEventRecord(ev[nev++], s));
    return KC_OK;
  };
  constexpr size_t N3 = (size_t)N * N * N;
  const size_t nbuf = (size_t)nvec * 3 * N3 * sizeof(cpx<T>);
  KC_TRY(op->work_a.ensure(nbuf));
  cpx<T>* A = op->work_a.as<cpx<T>>();
  const PassArgs<T> pa = pass_args<N, T>(op, ik0);
  const int* act = vm.active;
  if (op->scheme == KC_EPS_CROSSDOF) KC_TRY(op->work_b.ensure(nbuf));
  KC_TRY(op->work_k.ensure((size_t)nvec * N3 * sizeof(c64)));
  c64* kx = op->work_k.as<c64>();
  KC_TRY(mark());
  launch_x1<N, T, false>(op, TP_X1, nvec, x, A, pa.ktab, vm, pa.tw, s, nullptr, pa.ktab64, kx);
  KC_LAUNCHED();
  KC_TRY(mark());
  launch_y<N, +1, T>(op, TP_Y1, nvec, A, pa.tw, act, s);
  KC_LAUNCHED();
  KC_TRY(mark());
  if (op->scheme == KC_EPS_CROSSDOF) {
    cpx<T>* B = op->work_b.as<cpx<T>>();
    launch_zplain<N, +1, T>(op, TP_ZA, 3 * nvec, A, B, pa.tw, act, 3, s);
    KC_LAUNCHED();
    KC_TRY(mark());
    launch_zb<N, T>(op, nvec, B, A, pa.eps, pa.tw, act, s);
    KC_LAUNCHED();
  } else {
    launch_zt<N, T>(op, nvec, A, pa.eps, pa.tw, act, s);
    KC_LAUNCHED();
  }
  KC_TRY(mark());
  launch_y<N, -1, T>(op, TP_Y2, nvec, A, pa.tw, act, s);
  KC_LAUNCHED();
  KC_TRY(mark());
  launch_x2<N, T, false>(op, TP_X2, nvec, A, x, y, pa.ktab, pa.ktab64, pa.gam, vm, vm, pa.tw, s, nullptr, kx);
  KC_LAUNCHED();
  KC_TRY(mark());
  return KC_OK;
}

// y = T_E x (transverse-projection preconditioner); x is addressed through vm, y through vmy
// (same k-point grouping and active mask), and the two must not overlap.
template <int N, typename T>
static int apply_tp_n(kc_op* op, int ik0, int nvec, const VecMap& vm, const VecMap& vmy, const c64* x, c64* y,
                      const float* field, int fkstride, hipStream_t s, const double* sfl) {
  KC_TRY((tune_tiles_n<N, T>(op, nvec, s)));
  if (sfl) sfl += ik0;
  constexpr size_t N3 = (size_t)N * N * N;
  const size_t nbuf = (size_t)nvec * 3 * N3 * sizeof(cpx<T>);
  KC_TRY(op->work_a.ensure(nbuf));
  cpx<T>* A = op->work_a.as<cpx<T>>();
  const PassArgs<T> pa = pass_args<N, T>(op, ik0);
  const int* act = vm.active;
  if constexpr (plane_ok<N, T>()) {
    // fields with an x-major copy (the classical field shared by all k-points, the learned
    // fields one per k-point): x-passes in the x-major layout around one yz-plane pass
    const float* fieldt = nullptr;
    if (fkstride == 0 && field == op->efield.as<float>()) fieldt = op->efield_t.as<float>();
    if (fkstride == 1 && field == op->efield_k.as<float>()) fieldt = op->efield_kt.as<float>();
    if (fieldt != nullptr) {
      KC_TRY(op->work_k.ensure((size_t)nvec * N3 * sizeof(cpx<T>)));
      cpx<T>* kx = op->work_k.as<cpx<T>>();
      launch_x1<N, T, true, true>(op, TP_X1P, nvec, x, A, pa.ktab, vm, pa.tw, s, kx, nullptr, nullptr, sfl);
      KC_LAUNCHED();
      launch_yz<N, T>(nvec, A, fieldt, vm.vpk, fkstride, pa.tw, act, s);
      KC_LAUNCHED();
      launch_x2<N, T, true, true>(op, TP_X2P, nvec, A, x, y, pa.ktab, pa.ktab64, pa.gam, vm, vmy, pa.tw, s, kx,
                                  nullptr, sfl);
      KC_LAUNCHED();
      return KC_OK;
    }
  }
  launch_x1<N, T, true>(op, TP_X1P, nvec, x, A, pa.ktab, vm, pa.tw, s, nullptr, nullptr, nullptr, sfl);
  KC_LAUNCHED();
  launch_y<N, +1, T>(op, TP_Y1, nvec, A, pa.tw, act, s);
  KC_LAUNCHED();
  launch_zf<N, T>(op, nvec, A, field, vm.vpk, fkstride, pa.tw, act, s);
  KC_LAUNCHED();
  launch_y<N, -1, T>(op, TP_Y2, nvec, A, pa.tw, act, s);
  KC_LAUNCHED();
  launch_x2<N, T, true>(op, TP_X2P, nvec, A, x, y, pa.ktab, pa.ktab64, pa.gam, vm, vmy, pa.tw, s, nullptr, nullptr,
                        sfl);
  KC_LAUNCHED();
  return KC_OK;
}

// Times every candidate width of every pass on min(nvec, 32) vectors (inputs: the zero-filled
// work buffers; only the durations matter) and keeps the fastest per pass.  Runs once per
// handle and precision, never while the stream is being captured.
template <int N, typename T>
static int tune_tiles_n(kc_op* op, int nvec, hipStream_t s) {
  const int pi = sizeof(T) == 8 ? 1 : 0;
  if (op->tuned[pi]) return KC_OK;
  if (N < 32) {
    op->tuned[pi] = true;
    return KC_OK;
  }
  hipStreamCaptureStatus cs = hipStreamCaptureStatusNone;
  KC_HIP(hipStreamIsCapturing(s, &cs));
  if (cs != hipStreamCaptureStatusNone) return KC_OK;
  constexpr size_t N3 = (size_t)N * N * N;
  const int nv = std::max(1, std::min(nvec, 32));
  const size_t vb = (size_t)nv * 3 * N3;
  KC_TRY(op->work_a.ensure(vb * sizeof(c64)));
  KC_TRY(op->work_b.ensure(vb * sizeof(c64)));
  KC_TRY(op->work_c.ensure(2 * vb * sizeof(c64)));
  KC_TRY(op->work_k.ensure((size_t)nv * N3 * sizeof(c64)));
  KC_TRY(build_efield(op));
  cpx<T>* A = op->work_a.as<cpx<T>>();
  cpx<T>* B = op->work_b.as<cpx<T>>();
  c64* X = op->work_c.as<c64>();
  c64* Y = X + vb;
  const PassArgs<T> pa = pass_args<N, T>(op, 0);
  VecMap vm;
  vm.vpk = nv;
  vm.kstride = nv;
  const float* fld = op->efield.as<float>();
  hipEvent_t e0, e1;
  KC_HIP(hipEventCreate(&e0));
  KC_HIP(hipEventCreate(&e1));
  auto run_pass = [&](int pass) {
    switch (pass) {
      case TP_X1:
        launch_x1<N, T, false>(op, pass, nv, X, A, pa.ktab, vm, pa.tw, s, nullptr, pa.ktab64, op->work_k.as<c64>());
        break;
      case TP_X1P:
        launch_x1<N, T, true, plane_ok<N, T>()>(op, pass, nv, X, A, pa.ktab, vm, pa.tw, s, op->work_k.as<cpx<T>>());
        break;
      case TP_Y1: launch_y<N, +1, T>(op, pass, nv, A, pa.tw, nullptr, s); break;
      case TP_Y2: launch_y<N, -1, T>(op, pass, nv, A, pa.tw, nullptr, s); break;
      case TP_ZA: launch_zplain<N, +1, T>(op, pass, 3 * nv, A, B, pa.tw, nullptr, 3, s); break;
      case TP_ZB: launch_zb<N, T>(op, nv, B, A, pa.eps, pa.tw, nullptr, s); break;
      case TP_ZT: launch_zt<N, T>(op, nv, A, pa.eps, pa.tw, nullptr, s); break;
      case TP_ZF: launch_zf<N, T>(op, nv, A, fld, nv, 0, pa.tw, nullptr, s); break;
      case TP_X2:
        launch_x2<N, T, false>(op, pass, nv, A, X, Y, pa.ktab, pa.ktab64, pa.gam, vm, vm, pa.tw, s, nullptr,
                               op->work_k.as<c64>());
        break;
      case TP_X2P:
        launch_x2<N, T, true, plane_ok<N, T>()>(op, pass, nv, A, X, Y, pa.ktab, pa.ktab64, pa.gam, vm, vm, pa.tw, s,
                                                op->work_k.as<cpx<T>>());
        break;
      default: break;
    }
  };
  int st = KC_OK;
  for (int pass = 0; pass < TP_NPASS && st == KC_OK; ++pass) {
    const bool three = (pass == TP_X1 || pass == TP_X1P || pass == TP_X2 || pass == TP_X2P || pass == TP_ZB ||
                        pass == TP_ZT || pass == TP_ZF);
    const std::vector<int> cand = three ? tile_candidates<N, 3, T>() : tile_candidates<N, 1, T>();
    float best = 1e30f;
    int bestp = cand[0];
    for (int p : cand) {
      op->tiles[pi][pass] = (int8_t)p;
      run_pass(pass);  // warm-up
      hipError_t e = hipEventRecord(e0, s);
      for (int r = 0; r < 2 && e == hipSuccess; ++r) run_pass(pass);
      if (e == hipSuccess) e = hipEventRecord(e1, s);
      if (e == hipSuccess) e = hipGetLastError();
      if (e == hipSuccess) e = hipEventSynchronize(e1);
      float ms = 0.f;
      if (e == hipSuccess) e = hipEventElapsedTime(&ms, e0, e1);
      if (e != hipSuccess) {
        set_error(std::string("tile tuning: ") + hipGetErrorString(e));
        st = KC_ERR_HIP;
        break;
      }
      if (ms < best) {
        best = ms;
        bestp = p;
      }
    }
    op->tiles[pi][pass] = (int8_t)bestp;
  }
  (void)hipEventDestroy(e0);
  (void)hipEventDestroy(e1);
  if (st == KC_OK) op->tuned[pi] = true;
  return st;
}

// g[b][c][p] += sum_j w[b vpk + j] Re(conj(Ge_j) Gr_j)_c(p) with G = F3 K_A^{+} (the real-space
// edge field that T_E scales pointwise), for the vectors j of k-point group b: the gradient of
// sum_j w_j Re<e_j, T_E r_j> with respect to E.  Gr, Ge are unnormalised inverse DFTs, hence
// the factor 1/N^3.
template <typename T>
__global__ void k_tp_grad(const cpx<T>* __restrict__ Gr, const cpx<T>* __restrict__ Ge,
                          const double* __restrict__ w, int vpk, int nk, size_t N3, float* __restrict__ g) {
  const double inv = 1.0 / (double)N3;
  for (size_t t = (size_t)blockIdx.x * 256 + threadIdx.x; t < (size_t)nk * 3 * N3; t += (size_t)gridDim.x * 256) {
    const size_t b = t / (3 * N3), cp = t - b * 3 * N3;
    double acc = 0.0;
    for (int j = 0; j < vpk; ++j) {
      const size_t v = b * vpk + j;
      const cpx<T> a = Ge[v * 3 * N3 + cp], c = Gr[v * 3 * N3 + cp];
      acc += w[v] * (double)(a.re * c.re + a.im * c.im);
    }
    g[t] += (float)(acc * inv);
  }
}

template <int N>
static int tp_grad_n(kc_op* op, int ik0, int nvec, int vpk, const c64* r, const c64* e, const double* w, float* g,
                     hipStream_t s) {
  using T = double;
  constexpr size_t N3 = (size_t)N * N * N;
  const size_t nbuf = (size_t)nvec * 3 * N3 * sizeof(c64);
  KC_TRY(op->work_a.ensure(nbuf));
  KC_TRY(op->work_b.ensure(nbuf));
  KC_TRY(op->work_c.ensure(nbuf));
  c64* A = op->work_a.as<c64>();
  const PassArgs<T> pa = pass_args<N, T>(op, ik0);
  VecMap vm;
  vm.vpk = vpk;
  vm.kstride = vpk;
  c64* out[2] = {op->work_b.as<c64>(), op->work_c.as<c64>()};
  const c64* in[2] = {r, e};
  for (int i = 0; i < 2; ++i) {
    launch_x1<N, T, true>(op, TP_X1P, nvec, in[i], A, pa.ktab, vm, pa.tw, s);
    KC_LAUNCHED();
    launch_y<N, +1, T>(op, TP_Y1, nvec, A, pa.tw, nullptr, s);
    KC_LAUNCHED();
    launch_zplain<N, +1, T>(op, TP_ZA, 3 * nvec, A, out[i], pa.tw, nullptr, 3, s);
    KC_LAUNCHED();
  }
  const int nk = nvec / vpk;
  const unsigned gg = (unsigned)std::min<size_t>(((size_t)nk * 3 * N3 + 255) / 256, 65535);
  k_tp_grad<T><<<gg, 256, 0, s>>>(out[0], out[1], w, vpk, nk, N3, g);
  KC_LAUNCHED();
  return KC_OK;
}

// standalone 3D DFT (no handle): the default widths
template <int N, typename T>
static int fft3d_n(int nvec, int sign, const cpx<T>* in, cpx<T>* out, const cpx<T>* tw, hipStream_t s) {
  constexpr int P1 = TileP<N, 1, T>::P;
  const unsigned g1 = nblk((size_t)nvec * N * (N / P1));
  if (sign > 0) {
    k_x_plain<N, +1, T, P1><<<g1, NT, 0, s>>>(in, out, tw);
    KC_LAUNCHED();
    k_y<N, +1, T, P1><<<g1, NT, 0, s>>>(out, tw, nullptr);
    KC_LAUNCHED();
    k_z_plain<N, +1, T, P1><<<g1, NT, 0, s>>>(out, out, tw, nullptr, 1);
    KC_LAUNCHED();
  } else {
    k_x_plain<N, -1, T, P1><<<g1, NT, 0, s>>>(in, out, tw);
    KC_LAUNCHED();
    k_y<N, -1, T, P1><<<g1, NT, 0, s>>>(out, tw, nullptr);
    KC_LAUNCHED();
    k_z_plain<N, -1, T, P1><<<g1, NT, 0, s>>>(out, out, tw, nullptr, 1);
    KC_LAUNCHED();
  }
  return KC_OK;
}

#define KC_DISPATCH_N(N, CALL)                        \
  switch (N) {                                        \
    case 4: { constexpr int NN = 4; return CALL; }    \
    case 6: { constexpr int NN = 6; return CALL; }    \
    case 8: { constexpr int NN = 8; return CALL; }    \
    case 12: { constexpr int NN = 12; return CALL; }  \
    case 16: { constexpr int NN = 16; return CALL; }  \
    case 24: { constexpr int NN = 24; return CALL; }  \
    case 32: { constexpr int NN = 32; return CALL; }  \
    case 48: { constexpr int NN = 48; return CALL; }  \
    case 64: { constexpr int NN = 64; return CALL; }  \
    case 96: { constexpr int NN = 96; return CALL; }  \
    case 128: { constexpr int NN = 128; return CALL; } \
    default: break;                                   \
  }

template <int N>
static int prepare_n() {
  if constexpr (plane_ok<N, float>())
    KC_HIP(hipFuncSetAttribute((const void*)k_yz_field<N, float>, hipFuncAttributeMaxDynamicSharedMemorySize,
                               (int)plane_lds_bytes<N, float>()));
  return KC_OK;
}

int prepare_kernels(int N) {
  KC_DISPATCH_N(N, (prepare_n<NN>()))
  set_error("unsupported N");
  return KC_ERR_UNSUPPORTED;
}

int apply_op(kc_op* op, int ik0, int nvec, const VecMap& vm, const c64* x, c64* y, int prec, hipStream_t s,
             hipEvent_t* ev) {
  if (nvec == 0) return KC_OK;
  if (prec == KC_PREC_FP64) {
    KC_DISPATCH_N(op->N, (apply_n<NN, double>(op, ik0, nvec, vm, x, y, s, ev)))
  } else {
    KC_DISPATCH_N(op->N, (apply_n<NN, float>(op, ik0, nvec, vm, x, y, s, ev)))
  }
  set_error("unsupported N");
  return KC_ERR_UNSUPPORTED;
}

int apply_precond(kc_op* op, int ik0, int nvec, int vecs_per_k, const c64* r, c64* z, hipStream_t s) {
  if (nvec == 0) return KC_OK;
  const size_t tot = (size_t)op->N * op->N * op->N * nvec;
  const unsigned grid = (unsigned)std::min<size_t>((tot + NT - 1) / NT, 65536);
  k_precond<<<grid, NT, 0, s>>>(r, z, op->ktab64.as<c64>() + (size_t)ik0 * 3 * op->N, op->skew,
                                op->gamma_d.as<double>() + ik0, op->N, nvec, vecs_per_k);
  KC_LAUNCHED();
  return KC_OK;
}

int apply_tp(kc_op* op, int ik0, int nvec, const VecMap& vm, const VecMap& vmy, const c64* x, c64* y,
             const float* field, int fkstride, int prec, hipStream_t s, const double* sfl) {
  if (nvec == 0) return KC_OK;
  if (prec == KC_PREC_FP64) {
    KC_DISPATCH_N(op->N, (apply_tp_n<NN, double>(op, ik0, nvec, vm, vmy, x, y, field, fkstride, s, sfl)))
  } else {
    KC_DISPATCH_N(op->N, (apply_tp_n<NN, float>(op, ik0, nvec, vm, vmy, x, y, field, fkstride, s, sfl)))
  }
  set_error("unsupported N");
  return KC_ERR_UNSUPPORTED;
}

int tp_grad(kc_op* op, int ik0, int nvec, int vpk, const c64* r, const c64* e, const double* w, float* g,
            hipStream_t s) {
  if (nvec == 0) return KC_OK;
  KC_DISPATCH_N(op->N, (tp_grad_n<NN>(op, ik0, nvec, vpk, r, e, w, g, s)))
  set_error("unsupported N");
  return KC_ERR_UNSUPPORTED;
}

int fft3d(int N, int nvec, int sign, int prec, const void* in, void* out, const void* tw, hipStream_t s) {
  if (nvec == 0) return KC_OK;
  if (prec == KC_PREC_FP64) {
    KC_DISPATCH_N(N, (fft3d_n<NN, double>(nvec, sign, (const c64*)in, (c64*)out, (const c64*)tw, s)))
  } else {
    KC_DISPATCH_N(N, (fft3d_n<NN, float>(nvec, sign, (const c32*)in, (c32*)out, (const c32*)tw, s)))
  }
  set_error("unsupported N");
  return KC_ERR_UNSUPPORTED;
}

}  // namespace kc
