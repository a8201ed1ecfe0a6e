// LDS-resident pencil FFTs for gfx950.
//
// A workgroup holds a tile of NPEN pencils of length N in LDS and transforms all of them
// along their length with a Stockham autosort sequence of radix-R stages (R in {2,3,4,8,16}):
// at a stage with radix R after a sub-transform length NS, butterfly j of a pencil reads
// elements j + r N/R (r < R), multiplies them by exp(DIR 2 pi i r (j mod NS) / (NS R)),
// applies the length-R DFT and writes them to (j div NS) NS R + (j mod NS) + r NS.  After
// the last stage the pencil holds sum_j u_j exp(DIR 2 pi i j q / N) in natural order
// (unnormalised; DIR = +1 is the inverse direction of the unitary DFT of Lemma 2.1,
// DIR = -1 the forward direction).
//
// LDS layout of a tile: [c][element][pencil] with the pencil index fastest and a row pitch
// of P+1 (P pencils per component c).  Lanes are mapped pencil-fastest inside a stage, so
// reads and writes of a stage touch consecutive words whatever the FFT index pattern is;
// the odd pitch keeps element-fastest global->LDS transposes free of bank conflicts.
#pragma once

#include "kc_common.h"

namespace kc {

// radix plans (product = N); larger radices first
template <int N>
struct Plan;
#define KC_PLAN(n, s, r0, r1, r2)                       \
  template <>                                           \
  struct Plan<n> {                                      \
    static constexpr int S = s;                         \
    static constexpr int R[3] = {r0, r1, r2};           \
  };
KC_PLAN(4, 1, 4, 1, 1)
KC_PLAN(6, 2, 3, 2, 1)
KC_PLAN(8, 1, 8, 1, 1)
KC_PLAN(12, 2, 4, 3, 1)
KC_PLAN(16, 2, 4, 4, 1)
KC_PLAN(24, 2, 8, 3, 1)
KC_PLAN(32, 2, 8, 4, 1)
KC_PLAN(48, 3, 4, 4, 3)
KC_PLAN(64, 2, 8, 8, 1)
KC_PLAN(96, 3, 8, 4, 3)
KC_PLAN(128, 3, 8, 4, 4)
#undef KC_PLAN

// length-R DFT in registers: y_q = sum_r v_r exp(DIR 2 pi i r q / R)
template <int R, int DIR, typename T>
__device__ __forceinline__ void dft_small(cpx<T>* v);

template <int R, int DIR, typename T>
__device__ __forceinline__ void dft_small(cpx<T>* v) {
  if constexpr (R == 2) {
    cpx<T> a = v[0], b = v[1];
    v[0] = a + b;
    v[1] = a - b;
  } else if constexpr (R == 3) {
    const T h = static_cast<T>(0.5);
    const T s3 = static_cast<T>(DIR) * static_cast<T>(0.86602540378443864676372317075294);
    cpx<T> t1 = v[1] + v[2];
    cpx<T> t2 = v[1] - v[2];
    cpx<T> m = mk(v[0].re - h * t1.re, v[0].im - h * t1.im);
    cpx<T> j = mk(-s3 * t2.im, s3 * t2.re);  // DIR i sqrt(3)/2 t2
    v[0] = v[0] + t1;
    v[1] = m + j;
    v[2] = m - j;
  } else if constexpr (R == 4) {
    cpx<T> a = v[0] + v[2], b = v[0] - v[2];
    cpx<T> c = v[1] + v[3], d = v[1] - v[3];
    cpx<T> id = (DIR > 0) ? mul_i(d) : mk(d.im, -d.re);  // DIR i d
    v[0] = a + c;
    v[2] = a - c;
    v[1] = b + id;
    v[3] = b - id;
  } else if constexpr (R == 8) {
    cpx<T> e[4] = {v[0], v[2], v[4], v[6]};
    cpx<T> o[4] = {v[1], v[3], v[5], v[7]};
    dft_small<4, DIR, T>(e);
    dft_small<4, DIR, T>(o);
    const T r2 = static_cast<T>(0.70710678118654752440084436210485);
    // w8^q O_q, w8 = exp(DIR i pi/4)
    cpx<T> o1 = mk(r2 * (o[1].re - DIR * o[1].im), r2 * (o[1].im + DIR * o[1].re));
    cpx<T> o2 = (DIR > 0) ? mul_i(o[2]) : mk(o[2].im, -o[2].re);
    cpx<T> o3 = mk(r2 * (-o[3].re - DIR * o[3].im), r2 * (-o[3].im + DIR * o[3].re));
    v[0] = e[0] + o[0];
    v[4] = e[0] - o[0];
    v[1] = e[1] + o1;
    v[5] = e[1] - o1;
    v[2] = e[2] + o2;
    v[6] = e[2] - o2;
    v[3] = e[3] + o3;
    v[7] = e[3] - o3;
  } else if constexpr (R == 16) {
    // n = 4 n1 + n2, q = q1 + 4 q2: length-4 DFTs over n1, twiddles w16^(n2 q1), length-4 DFTs
    // over n2 (w16 = exp(DIR i pi/8))
    const T c1 = static_cast<T>(0.92387953251128675613), s1 = static_cast<T>(0.38268343236508977173);
    const T r2 = static_cast<T>(0.70710678118654752440);
    const T d = static_cast<T>(DIR);
    const cpx<T> w[10] = {mk(T(1), T(0)),  mk(c1, d * s1),   mk(r2, d * r2),   mk(s1, d * c1),
                          mk(T(0), d),     mk(-s1, d * c1),  mk(-r2, d * r2),  mk(-c1, d * s1),
                          mk(T(-1), T(0)), mk(-c1, -d * s1)};
    cpx<T> a[4][4];
#pragma unroll
    for (int n2 = 0; n2 < 4; ++n2) {
#pragma unroll
      for (int n1 = 0; n1 < 4; ++n1) a[n2][n1] = v[4 * n1 + n2];
      dft_small<4, DIR, T>(a[n2]);  // a[n2][q1]
#pragma unroll
      for (int q1 = 1; q1 < 4; ++q1)
        if (n2 > 0) a[n2][q1] = a[n2][q1] * w[n2 * q1];
    }
#pragma unroll
    for (int q1 = 0; q1 < 4; ++q1) {
      cpx<T> b[4] = {a[0][q1], a[1][q1], a[2][q1], a[3][q1]};
      dft_small<4, DIR, T>(b);
#pragma unroll
      for (int q2 = 0; q2 < 4; ++q2) v[q1 + 4 * q2] = b[q2];
    }
  }
}

// Tile geometry: NC components x P pencils, each of N elements; pitch P+1.
template <int N, int P, int NC>
struct TileGeom {
  static constexpr int PP = P + 1;
  static constexpr int CSTRIDE = N * PP;
  static constexpr int ELEMS = NC * CSTRIDE;  // LDS elements
  static constexpr int NPEN = NC * P;
  __device__ static __forceinline__ int addr(int pen, int e) {
    const int c = pen / P;
    const int p = pen - c * P;
    return c * CSTRIDE + e * PP + p;
  }
  __device__ static __forceinline__ int addr3(int c, int e, int p) { return c * CSTRIDE + e * PP + p; }
};

// twiddle table tw[t] = exp(+2 pi i t / N), t < N, staged in LDS by the caller
template <int N, typename T>
__device__ __forceinline__ void load_twiddles(cpx<T>* tw, const cpx<T>* gtw) {
  for (int t = threadIdx.x; t < N; t += blockDim.x) tw[t] = gtw[t];
}

template <int N, int P, int NC, int NT, int R, int NS, int DIR, typename T>
__device__ __forceinline__ void fft_stage(cpx<T>* lds, const cpx<T>* tw) {
  using G = TileGeom<N, P, NC>;
  constexpr int NB = N / R;
  constexpr int TOT = G::NPEN * NB;
  constexpr int IT = (TOT + NT - 1) / NT;
  const int tid = threadIdx.x;
  cpx<T> v[IT][R];
#pragma unroll
  for (int it = 0; it < IT; ++it) {
    const int w = tid + it * NT;
    if ((TOT % NT) == 0 || w < TOT) {
      const int pen = w % G::NPEN;
      const int j = w / G::NPEN;
#pragma unroll
      for (int r = 0; r < R; ++r) v[it][r] = lds[G::addr(pen, j + r * NB)];
    }
  }
  __syncthreads();
#pragma unroll
  for (int it = 0; it < IT; ++it) {
    const int w = tid + it * NT;
    if ((TOT % NT) == 0 || w < TOT) {
      const int pen = w % G::NPEN;
      const int j = w / G::NPEN;
      const int k = j % NS;
      if constexpr (NS > 1) {
        constexpr int STEP = N / (NS * R);
#pragma unroll
        for (int r = 1; r < R; ++r) {
          cpx<T> t = tw[r * k * STEP];
          if (DIR < 0) t.im = -t.im;
          v[it][r] = v[it][r] * t;
        }
      }
      dft_small<R, DIR, T>(v[it]);
      const int base = (j / NS) * NS * R + k;
#pragma unroll
      for (int r = 0; r < R; ++r) lds[G::addr(pen, base + r * NS)] = v[it][r];
    }
  }
  __syncthreads();
}

template <int N, int P, int NC, int NT, int DIR, typename T, int S = 0, int NS = 1>
__device__ __forceinline__ void fft_tile(cpx<T>* lds, const cpx<T>* tw) {
  if constexpr (S < Plan<N>::S) {
    constexpr int R = Plan<N>::R[S];
    fft_stage<N, P, NC, NT, R, NS, DIR, T>(lds, tw);
    fft_tile<N, P, NC, NT, DIR, T, S + 1, NS * R>(lds, tw);
  }
}

// The same stages on a 2D tile: NPEN pencils of N elements at lds[pen * PS + e * ES] (one of
// PS, ES is 1, the other the row pitch).  Lanes run pencil-fastest: along a column (PS == 1)
// the accesses are consecutive words, along a row (ES == 1) they are one pitch apart, which an
// odd pitch spreads over the banks.
template <int N, int NPEN, int ES, int PS, int NTH, int R, int NS, int DIR, typename T>
__device__ __forceinline__ void fft_stage_2d(cpx<T>* lds, const cpx<T>* tw) {
  constexpr int NB = N / R;
  constexpr int TOT = NPEN * NB;
  constexpr int IT = (TOT + NTH - 1) / NTH;
  const int tid = threadIdx.x;
  cpx<T> v[IT][R];
#pragma unroll
  for (int it = 0; it < IT; ++it) {
    const int w = tid + it * NTH;
    if ((TOT % NTH) == 0 || w < TOT) {
      const int pen = w % NPEN, j = w / NPEN;
#pragma unroll
      for (int r = 0; r < R; ++r) v[it][r] = lds[pen * PS + (j + r * NB) * ES];
    }
  }
  __syncthreads();
#pragma unroll
  for (int it = 0; it < IT; ++it) {
    const int w = tid + it * NTH;
    if ((TOT % NTH) == 0 || w < TOT) {
      const int pen = w % NPEN, j = w / NPEN;
      const int k = j % NS;
      if constexpr (NS > 1) {
        constexpr int STEP = N / (NS * R);
#pragma unroll
        for (int r = 1; r < R; ++r) {
          cpx<T> t = tw[r * k * STEP];
          if (DIR < 0) t.im = -t.im;
          v[it][r] = v[it][r] * t;
        }
      }
      dft_small<R, DIR, T>(v[it]);
      const int base = (j / NS) * NS * R + k;
#pragma unroll
      for (int r = 0; r < R; ++r) lds[pen * PS + (base + r * NS) * ES] = v[it][r];
    }
  }
  __syncthreads();
}

// radix plans of the 2D tiles (one butterfly per thread at N = 128 and 1024 threads, so the
// larger radix costs no extra registers and saves a stage per direction)
template <int N>
struct Plan2D : Plan<N> {};
template <>
struct Plan2D<128> {
  static constexpr int S = 2;
  static constexpr int R[3] = {16, 8, 1};
};

template <int N, int NPEN, int ES, int PS, int NTH, int DIR, typename T, int S = 0, int NS = 1>
__device__ __forceinline__ void fft_2d(cpx<T>* lds, const cpx<T>* tw) {
  if constexpr (S < Plan2D<N>::S) {
    constexpr int R = Plan2D<N>::R[S];
    fft_stage_2d<N, NPEN, ES, PS, NTH, R, NS, DIR, T>(lds, tw);
    fft_2d<N, NPEN, ES, PS, NTH, DIR, T, S + 1, NS * R>(lds, tw);
  }
}

}  // namespace kc
