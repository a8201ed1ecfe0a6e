// Matrix-free application of the kernel-compensated operator in k-space (Prop 2.8,
// eq (2.30)) and of the diagonal-block preconditioner (eqs (2.31)-(2.32)) on gfx950.
//
// y = K_A F3^H M F3 K_A^H x + gamma K_B x is evaluated in pencil passes over the
// [vec][3][z][y][x] layout, each pass one round trip of the block through HBM:
//
//   X1  e = -conj(K) x x (curl symbol, prologue), inverse DFT along x         (3 comps)
//   Y1  inverse DFT along y                                                   (per comp)
//   Z   Trivial/diagonal: inverse DFT along z, E' = M E / N^3 pointwise,
//       forward DFT along z                                                   (3 comps)
//       CrossDoF: Za inverse DFT along z (per comp); Zb E' = M E / N^3 with the
//       four-point cross-DoF averages read around each point, forward DFT along z
//   Y2  forward DFT along y                                                   (per comp)
//   X2  forward DFT along x, y = K x e' + gamma conj(K) (K . x) (epilogue, re-reads x)
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
// singular, and equals K_P^{-1} for E = 1.
#include <algorithm>
#include <cmath>

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
// X1: curl prologue + inverse DFT along x.  Tile: P rows (y) of one (vec, z), 3 comps.
// ------------------------------------------------------------------------------------
template <int N, typename T, bool PRE>
__global__ __launch_bounds__(NT) void k_x1_curl_inv(const c64* __restrict__ x, cpx<T>* __restrict__ E,
                                                    const cpx<T>* __restrict__ ktab, VecMap vm,
                                                    const cpx<T>* __restrict__ gtw) {
  constexpr int P = TileP<N, 3, T>::P;
  using G = TileGeom<N, P, 3>;
  __shared__ cpx<T> lds[G::ELEMS];
  __shared__ cpx<T> tw[N];
  constexpr size_t N3 = (size_t)N * N * N;
  unsigned b = blockIdx.x;
  const int yt = b % (N / P);
  b /= (N / P);
  const int z = b % N;
  const int vec = b / N;
  if (!vm.on(vec)) return;
  const cpx<T>* K = ktab + (size_t)(vec / vm.vpk) * 3 * N;
  load_twiddles<N>(tw, gtw);
  const c64* xv = x + vm.off(vec) * 3 * N3;
  const cpx<T> v3 = conj(K[2 * N + z]);
  for (int w = threadIdx.x; w < N * P; w += NT) {
    const int e = w % N, p = w / N, y = yt * P + p;
    const size_t off = (size_t)z * N * N + (size_t)y * N + e;
    const cpx<T> x1 = cvt<T>(xv[off]), x2 = cvt<T>(xv[N3 + off]), x3 = cvt<T>(xv[2 * N3 + off]);
    const cpx<T> v1 = conj(K[e]), v2 = conj(K[N + y]);
    cpx<T> c1 = v3 * x2 - v2 * x3, c2 = v1 * x3 - v3 * x1, c3 = v2 * x1 - v1 * x2;
    if (PRE) {  // K_A^{+} = K_A^H / s
      const T sq = abs2(v1) + abs2(v2) + abs2(v3);
      const T is = sq > T(0) ? T(1) / sq : T(0);
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
  for (int w = threadIdx.x; w < 3 * N * P; w += NT) {
    const int e = w % N, p = (w / N) % P, c = w / (N * P), y = yt * P + p;
    Ev[c * N3 + (size_t)z * N * N + (size_t)y * N + e] = lds[G::addr3(c, e, p)];
  }
}

// ------------------------------------------------------------------------------------
// X2: forward DFT along x + outer curl + penalty epilogue.
// ------------------------------------------------------------------------------------
template <int N, typename T, bool PRE>
__global__ __launch_bounds__(NT) void k_x2_fwd_curl_pen(const cpx<T>* __restrict__ E,
                                                        const c64* __restrict__ x, c64* __restrict__ y,
                                                        const cpx<T>* __restrict__ ktab,
                                                        const c64* __restrict__ ktab64,
                                                        const double* __restrict__ gamma,
                                                        VecMap vm, VecMap vmy, const cpx<T>* __restrict__ gtw) {
  constexpr int P = TileP<N, 3, T>::P;
  using G = TileGeom<N, P, 3>;
  __shared__ cpx<T> lds[G::ELEMS];
  __shared__ cpx<T> tw[N];
  constexpr size_t N3 = (size_t)N * N * N;
  unsigned b = blockIdx.x;
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
  for (int w = threadIdx.x; w < 3 * N * P; w += NT) {
    const int e = w % N, p = (w / N) % P, c = w / (N * P), yy = yt * P + p;
    lds[G::addr3(c, e, p)] = Ev[c * N3 + (size_t)z * N * N + (size_t)yy * N + e];
  }
  __syncthreads();
  fft_tile<N, P, 3, NT, -1, T>(lds, tw);
  const c64* xv = x + vm.off(vec) * 3 * N3;
  c64* yv = y + vmy.off(vec) * 3 * N3;
  const cpx<T> K3 = K[2 * N + z];
  const c64 K3d = Kd[2 * N + z];
  for (int w = threadIdx.x; w < N * P; w += NT) {
    const int e = w % N, p = w / N, yy = yt * P + p;
    const size_t off = (size_t)z * N * N + (size_t)yy * N + e;
    const cpx<T> e1 = lds[G::addr3(0, e, p)], e2 = lds[G::addr3(1, e, p)], e3 = lds[G::addr3(2, e, p)];
    const cpx<T> K1 = K[e], K2 = K[N + yy];
    const c64 c1 = cvt<double>(K2 * e3 - K3 * e2);
    const c64 c2 = cvt<double>(K3 * e1 - K1 * e3);
    const c64 c3 = cvt<double>(K1 * e2 - K2 * e1);
    const c64 x1 = xv[off], x2 = xv[N3 + off], x3 = xv[2 * N3 + off];
    const c64 K1d = Kd[e], K2d = Kd[N + yy];
    const c64 kx = K1d * x1 + K2d * x2 + K3d * x3;  // K . x
    if (PRE) {  // (1/s) [c + (1/gamma) K_B x / s]
      const double sq = abs2(K1d) + abs2(K2d) + abs2(K3d);
      const double is = sq > 0.0 ? 1.0 / sq : 0.0;
      const c64 gk = (g * is) * kx;
      yv[off] = is * (c1 + cmulc(K1d, gk));
      yv[N3 + off] = is * (c2 + cmulc(K2d, gk));
      yv[2 * N3 + off] = is * (c3 + cmulc(K3d, gk));
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
template <int N, int DIR, typename T>
__global__ __launch_bounds__(NT) void k_y(cpx<T>* __restrict__ buf, const cpx<T>* __restrict__ gtw,
                                          const int* __restrict__ active) {
  constexpr int P = TileP<N, 1, T>::P;
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
template <int N, int DIR, typename T>
__global__ __launch_bounds__(NT) void k_x_plain(const cpx<T>* in, cpx<T>* out, const cpx<T>* __restrict__ gtw) {
  constexpr int P = TileP<N, 1, T>::P;
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
template <int N, int DIR, typename T>
__global__ __launch_bounds__(NT) void k_z_plain(const cpx<T>* in, cpx<T>* out, const cpx<T>* __restrict__ gtw,
                                                const int* __restrict__ active, int ncomp) {
  constexpr int P = TileP<N, 1, T>::P;
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
template <int N, typename T>
__global__ __launch_bounds__(NT) void k_z_trivial(cpx<T>* __restrict__ buf, const uint32_t* __restrict__ ids,
                                                  const EpsEntry<T>* __restrict__ geps, int n_mat,
                                                  const cpx<T>* __restrict__ gtw, const int* __restrict__ active) {
  constexpr int P = TileP<N, 3, T>::P;
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
template <int N, typename T>
__global__ __launch_bounds__(NT) void k_z_field(cpx<T>* __restrict__ buf, const float* __restrict__ field,
                                                int vpk, int fkstride, const cpx<T>* __restrict__ gtw,
                                                const int* __restrict__ active) {
  constexpr int P = TileP<N, 3, T>::P;
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
// Zb (CrossDoF): E' = M_CrossDoF E / N^3 (eq (3.8)) evaluated around each point from the
// real-space field E, then forward DFT along z.  With Q^(e)_cd the (c,d) entry of the
// inverse permittivity at the e-edge points and T_cd the four-point averages of eq (3.7),
// block (c,d), c < d, is (Q^(c)_cd T_cd + T_cd Q^(d)_cd)/2, so at a point P
//   [block(c,d) E_d](P) = 1/8 sum_{S in T_cd-stencil(P)} (Q^(c)_cd(P) + Q^(d)_cd(S)) E_d(S)
// and the lower blocks are the conjugate transposes.  Stencils (0-based, periodic):
//   T12: (i,j),(i-1,j),(i,j+1),(i-1,j+1)   T13: (i,k),(i-1,k),(i,k+1),(i-1,k+1)
//   T23: (j,k),(j-1,k),(j,k+1),(j-1,k+1)   and their transposes mirrored.
// Tile: P consecutive x of one (vec, y), 3 comps; E is read around the tile through the cache.
// ------------------------------------------------------------------------------------
template <typename T>
struct CrossCtx {
  const cpx<T>* E1;
  const cpx<T>* E2;
  const cpx<T>* E3;
  const uint32_t* ids;
  const EpsEntry<T>* eps;
  int N;
  __device__ __forceinline__ size_t at(int i, int j, int k) const {
    return ((size_t)k * N + j) * N + i;
  }
};

template <typename T>
__device__ __forceinline__ void crossdof_point(const CrossCtx<T>& C, int i, int j, int k, cpx<T>& o1,
                                               cpx<T>& o2, cpx<T>& o3) {
  const int N = C.N;
  const int ip = (i + 1 == N) ? 0 : i + 1, im = (i == 0) ? N - 1 : i - 1;
  const int jp = (j + 1 == N) ? 0 : j + 1, jm = (j == 0) ? N - 1 : j - 1;
  const int kp = (k + 1 == N) ? 0 : k + 1, km = (k == 0) ? N - 1 : k - 1;
  const size_t c0 = C.at(i, j, k);
  const uint32_t idc = C.ids[c0];
  const EpsEntry<T>& ex = C.eps[idc & 255u];
  const EpsEntry<T>& ey = C.eps[(idc >> 8) & 255u];
  const EpsEntry<T>& ez = C.eps[(idc >> 16) & 255u];
  const T e8 = static_cast<T>(0.125);
  auto mx = [&](size_t a) -> const EpsEntry<T>& { return C.eps[C.ids[a] & 255u]; };
  auto my = [&](size_t a) -> const EpsEntry<T>& { return C.eps[(C.ids[a] >> 8) & 255u]; };
  auto mz = [&](size_t a) -> const EpsEntry<T>& { return C.eps[(C.ids[a] >> 16) & 255u]; };

  // row 1: d1 E1 + block(1,2) E2 + block(1,3) E3
  cpx<T> a1 = mk<T>(0, 0);
  {
    const size_t s[4] = {c0, C.at(im, j, k), C.at(i, jp, k), C.at(im, jp, k)};
#pragma unroll
    for (int t = 0; t < 4; ++t) a1 = a1 + (ex.o[0] + my(s[t]).o[0]) * C.E2[s[t]];
  }
  {
    const size_t s[4] = {c0, C.at(im, j, k), C.at(i, j, kp), C.at(im, j, kp)};
#pragma unroll
    for (int t = 0; t < 4; ++t) a1 = a1 + (ex.o[1] + mz(s[t]).o[1]) * C.E3[s[t]];
  }
  o1 = ex.d[0] * C.E1[c0] + e8 * a1;

  // row 2: block(2,1) E1 + d2 E2 + block(2,3) E3
  cpx<T> a2 = mk<T>(0, 0);
  {
    const size_t s[4] = {c0, C.at(ip, j, k), C.at(i, jm, k), C.at(ip, jm, k)};
#pragma unroll
    for (int t = 0; t < 4; ++t) a2 = a2 + cmulc(mx(s[t]).o[0] + ey.o[0], C.E1[s[t]]);
  }
  {
    const size_t s[4] = {c0, C.at(i, jm, k), C.at(i, j, kp), C.at(i, jm, kp)};
#pragma unroll
    for (int t = 0; t < 4; ++t) a2 = a2 + (ey.o[2] + mz(s[t]).o[2]) * C.E3[s[t]];
  }
  o2 = ey.d[1] * C.E2[c0] + e8 * a2;

  // row 3: block(3,1) E1 + block(3,2) E2 + d3 E3
  cpx<T> a3 = mk<T>(0, 0);
  {
    const size_t s[4] = {c0, C.at(ip, j, k), C.at(i, j, km), C.at(ip, j, km)};
#pragma unroll
    for (int t = 0; t < 4; ++t) a3 = a3 + cmulc(mx(s[t]).o[1] + ez.o[1], C.E1[s[t]]);
  }
  {
    const size_t s[4] = {c0, C.at(i, jp, k), C.at(i, j, km), C.at(i, jp, km)};
#pragma unroll
    for (int t = 0; t < 4; ++t) a3 = a3 + cmulc(my(s[t]).o[2] + ez.o[2], C.E2[s[t]]);
  }
  o3 = ez.d[2] * C.E3[c0] + e8 * a3;
}

template <int N, typename T>
__global__ __launch_bounds__(NT) void k_zb_crossdof(const cpx<T>* __restrict__ E, cpx<T>* __restrict__ out,
                                                    const uint32_t* __restrict__ ids,
                                                    const EpsEntry<T>* __restrict__ geps, int n_mat,
                                                    const cpx<T>* __restrict__ gtw, const int* __restrict__ active) {
  constexpr int P = TileP<N, 3, T>::P;
  using G = TileGeom<N, P, 3>;
  __shared__ cpx<T> lds[G::ELEMS];
  __shared__ cpx<T> tw[N];
  __shared__ EpsEntry<T> eps[KC_MAX_MAT];
  constexpr size_t N3 = (size_t)N * N * N;
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
  CrossCtx<T> C;
  C.E1 = E + vec * 3 * N3;
  C.E2 = C.E1 + N3;
  C.E3 = C.E2 + N3;
  C.ids = ids;
  C.eps = eps;
  C.N = N;
  for (int w = threadIdx.x; w < N * P; w += NT) {
    const int p = w % P, e = w / P;
    cpx<T> o1, o2, o3;
    crossdof_point(C, xt * P + p, yy, e, o1, o2, o3);
    lds[G::addr3(0, e, p)] = o1;
    lds[G::addr3(1, e, p)] = o2;
    lds[G::addr3(2, e, p)] = o3;
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
__global__ __launch_bounds__(NT) void k_precond(const c64* r, c64* z, const c64* __restrict__ ktab64,
                                                const double* __restrict__ gamma, int N, int nvec,
                                                int vecs_per_k) {
  const size_t N3 = (size_t)N * N * N;
  const size_t tot = N3 * nvec;
  for (size_t t = (size_t)blockIdx.x * NT + threadIdx.x; t < tot; t += (size_t)gridDim.x * NT) {
    const size_t vec = t / N3, p = t - vec * N3;
    const int ik = (int)(vec / vecs_per_k);
    const c64* K = ktab64 + (size_t)ik * 3 * N;
    const int qx = (int)(p % N), qy = (int)((p / N) % N), qz = (int)(p / ((size_t)N * N));
    const c64 K1 = K[qx], K2 = K[N + qy], K3 = K[2 * N + qz];
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

template <int N, typename T>
static int apply_n(kc_op* op, int ik0, int nvec, const VecMap& vm, const c64* x, c64* y, hipStream_t s,
                   hipEvent_t* ev) {
  int nev = 0;
  auto mark = [&]() -> int {
    if (ev) KC_HIP(hipEventRecord(ev[nev++], s));
    return KC_OK;
  };
  constexpr size_t N3 = (size_t)N * N * N;
  const size_t nbuf = (size_t)nvec * 3 * N3 * sizeof(cpx<T>);
  KC_TRY(op->work_a.ensure(nbuf));
  cpx<T>* A = op->work_a.as<cpx<T>>();
  const bool f64 = sizeof(T) == 8;
  const cpx<T>* ktab = (f64 ? op->ktab64.as<cpx<T>>() : op->ktab32.as<cpx<T>>()) + (size_t)ik0 * 3 * N;
  const c64* ktab64 = op->ktab64.as<c64>() + (size_t)ik0 * 3 * N;
  const double* gam = op->gamma_d.as<double>() + ik0;
  const cpx<T>* tw = f64 ? op->tw64.as<cpx<T>>() : op->tw32.as<cpx<T>>();
  const EpsEntry<T>* eps = f64 ? op->eps64.as<EpsEntry<T>>() : op->eps32.as<EpsEntry<T>>();
  const uint32_t* ids = op->ids.as<uint32_t>();
  constexpr int P3 = TileP<N, 3, T>::P;
  constexpr int P1 = TileP<N, 1, T>::P;
  const unsigned g3 = nblk((size_t)nvec * N * (N / P3));
  const unsigned g1 = nblk((size_t)nvec * 3 * N * (N / P1));
  const int* act = vm.active;
  if (op->scheme == KC_EPS_CROSSDOF) KC_TRY(op->work_b.ensure(nbuf));
  KC_TRY(mark());
  k_x1_curl_inv<N, T, false><<<g3, NT, 0, s>>>(x, A, ktab, vm, tw);
  KC_LAUNCHED();
  KC_TRY(mark());
  k_y<N, +1, T><<<g1, NT, 0, s>>>(A, tw, act);
  KC_LAUNCHED();
  KC_TRY(mark());
  if (op->scheme == KC_EPS_CROSSDOF) {
    cpx<T>* B = op->work_b.as<cpx<T>>();
    k_z_plain<N, +1, T><<<g1, NT, 0, s>>>(A, B, tw, act, 3);
    KC_LAUNCHED();
    KC_TRY(mark());
    k_zb_crossdof<N, T><<<g3, NT, 0, s>>>(B, A, ids, eps, op->n_mat, tw, act);
    KC_LAUNCHED();
  } else {
    k_z_trivial<N, T><<<g3, NT, 0, s>>>(A, ids, eps, op->n_mat, tw, act);
    KC_LAUNCHED();
  }
  KC_TRY(mark());
  k_y<N, -1, T><<<g1, NT, 0, s>>>(A, tw, act);
  KC_LAUNCHED();
  KC_TRY(mark());
  k_x2_fwd_curl_pen<N, T, false><<<g3, NT, 0, s>>>(A, x, y, ktab, ktab64, gam, vm, vm, tw);
  KC_LAUNCHED();
  KC_TRY(mark());
  return KC_OK;
}

// y = T_E x (transverse-projection preconditioner); x is addressed through vm, y through vmy
// (same k-point grouping and active mask), and the two must not overlap.
template <int N, typename T>
static int apply_tp_n(kc_op* op, int ik0, int nvec, const VecMap& vm, const VecMap& vmy, const c64* x, c64* y,
                      const float* field, int fkstride, hipStream_t s) {
  constexpr size_t N3 = (size_t)N * N * N;
  const size_t nbuf = (size_t)nvec * 3 * N3 * sizeof(cpx<T>);
  KC_TRY(op->work_a.ensure(nbuf));
  cpx<T>* A = op->work_a.as<cpx<T>>();
  const bool f64 = sizeof(T) == 8;
  const cpx<T>* ktab = (f64 ? op->ktab64.as<cpx<T>>() : op->ktab32.as<cpx<T>>()) + (size_t)ik0 * 3 * N;
  const c64* ktab64 = op->ktab64.as<c64>() + (size_t)ik0 * 3 * N;
  const double* gam = op->gamma_d.as<double>() + ik0;
  const cpx<T>* tw = f64 ? op->tw64.as<cpx<T>>() : op->tw32.as<cpx<T>>();
  constexpr int P3 = TileP<N, 3, T>::P;
  constexpr int P1 = TileP<N, 1, T>::P;
  const unsigned g3 = nblk((size_t)nvec * N * (N / P3));
  const unsigned g1 = nblk((size_t)nvec * 3 * N * (N / P1));
  const int* act = vm.active;
  k_x1_curl_inv<N, T, true><<<g3, NT, 0, s>>>(x, A, ktab, vm, tw);
  KC_LAUNCHED();
  k_y<N, +1, T><<<g1, NT, 0, s>>>(A, tw, act);
  KC_LAUNCHED();
  k_z_field<N, T><<<g3, NT, 0, s>>>(A, field, vm.vpk, fkstride, tw, act);
  KC_LAUNCHED();
  k_y<N, -1, T><<<g1, NT, 0, s>>>(A, tw, act);
  KC_LAUNCHED();
  k_x2_fwd_curl_pen<N, T, true><<<g3, NT, 0, s>>>(A, x, y, ktab, ktab64, gam, vm, vmy, tw);
  KC_LAUNCHED();
  return KC_OK;
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
  const c64* ktab = op->ktab64.as<c64>() + (size_t)ik0 * 3 * N;
  const c64* tw = op->tw64.as<c64>();
  constexpr int P3 = TileP<N, 3, T>::P;
  constexpr int P1 = TileP<N, 1, T>::P;
  const unsigned g3 = nblk((size_t)nvec * N * (N / P3));
  const unsigned g1 = nblk((size_t)nvec * 3 * N * (N / P1));
  VecMap vm;
  vm.vpk = vpk;
  vm.kstride = vpk;
  c64* out[2] = {op->work_b.as<c64>(), op->work_c.as<c64>()};
  const c64* in[2] = {r, e};
  for (int i = 0; i < 2; ++i) {
    k_x1_curl_inv<N, T, true><<<g3, NT, 0, s>>>(in[i], A, ktab, vm, tw);
    KC_LAUNCHED();
    k_y<N, +1, T><<<g1, NT, 0, s>>>(A, tw, nullptr);
    KC_LAUNCHED();
    k_z_plain<N, +1, T><<<g1, NT, 0, s>>>(A, out[i], tw, nullptr, 3);
    KC_LAUNCHED();
  }
  const int nk = nvec / vpk;
  const unsigned gg = (unsigned)std::min<size_t>(((size_t)nk * 3 * N3 + 255) / 256, 65535);
  k_tp_grad<T><<<gg, 256, 0, s>>>(out[0], out[1], w, vpk, nk, N3, g);
  KC_LAUNCHED();
  return KC_OK;
}

template <int N, typename T>
static int fft3d_n(int nvec, int sign, const cpx<T>* in, cpx<T>* out, const cpx<T>* tw, hipStream_t s) {
  constexpr int P1 = TileP<N, 1, T>::P;
  const unsigned g1 = nblk((size_t)nvec * N * (N / P1));
  if (sign > 0) {
    k_x_plain<N, +1, T><<<g1, NT, 0, s>>>(in, out, tw);
    KC_LAUNCHED();
    k_y<N, +1, T><<<g1, NT, 0, s>>>(out, tw, nullptr);
    KC_LAUNCHED();
    k_z_plain<N, +1, T><<<g1, NT, 0, s>>>(out, out, tw, nullptr, 1);
    KC_LAUNCHED();
  } else {
    k_x_plain<N, -1, T><<<g1, NT, 0, s>>>(in, out, tw);
    KC_LAUNCHED();
    k_y<N, -1, T><<<g1, NT, 0, s>>>(out, tw, nullptr);
    KC_LAUNCHED();
    k_z_plain<N, -1, T><<<g1, NT, 0, s>>>(out, out, tw, nullptr, 1);
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
  k_precond<<<grid, NT, 0, s>>>(r, z, op->ktab64.as<c64>() + (size_t)ik0 * 3 * op->N,
                                op->gamma_d.as<double>() + ik0, op->N, nvec, vecs_per_k);
  KC_LAUNCHED();
  return KC_OK;
}

int apply_tp(kc_op* op, int ik0, int nvec, const VecMap& vm, const VecMap& vmy, const c64* x, c64* y,
             const float* field, int fkstride, int prec, hipStream_t s) {
  if (nvec == 0) return KC_OK;
  if (prec == KC_PREC_FP64) {
    KC_DISPATCH_N(op->N, (apply_tp_n<NN, double>(op, ik0, nvec, vm, vmy, x, y, field, fkstride, s)))
  } else {
    KC_DISPATCH_N(op->N, (apply_tp_n<NN, float>(op, ik0, nvec, vm, vmy, x, y, field, fkstride, s)))
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
