// Common definitions of the kcpc HIP library (gfx950): complex type, error plumbing,
// launch helpers.
#pragma once

#include <hip/hip_runtime.h>

#include <cstddef>
#include <cstdint>
#include <string>

#include "../../include/kcpc.h"

namespace kc {

// ----------------------------------------------------------------------------------------
// complex numbers: interleaved (re, im), 8- or 16-byte aligned so a load is one vector op
// ----------------------------------------------------------------------------------------
template <typename T>
struct alignas(2 * sizeof(T)) cpx {
  T re, im;
};

template <typename T>
__host__ __device__ __forceinline__ cpx<T> mk(T r, T i) {
  cpx<T> z;
  z.re = r;
  z.im = i;
  return z;
}
template <typename T>
__host__ __device__ __forceinline__ cpx<T> operator+(cpx<T> a, cpx<T> b) {
  return mk(a.re + b.re, a.im + b.im);
}
template <typename T>
__host__ __device__ __forceinline__ cpx<T> operator-(cpx<T> a, cpx<T> b) {
  return mk(a.re - b.re, a.im - b.im);
}
template <typename T>
__host__ __device__ __forceinline__ cpx<T> operator*(cpx<T> a, cpx<T> b) {
  return mk(a.re * b.re - a.im * b.im, a.re * b.im + a.im * b.re);
}
template <typename T>
__host__ __device__ __forceinline__ cpx<T> operator*(T s, cpx<T> a) {
  return mk(s * a.re, s * a.im);
}
template <typename T>
__host__ __device__ __forceinline__ cpx<T> conj(cpx<T> a) {
  return mk(a.re, -a.im);
}
// conj(a) * b
template <typename T>
__host__ __device__ __forceinline__ cpx<T> cmulc(cpx<T> a, cpx<T> b) {
  return mk(a.re * b.re + a.im * b.im, a.re * b.im - a.im * b.re);
}

// acc += a b and acc += conj(a) b as four fused multiply-adds (no separate product and sum)
template <typename T>
__device__ __forceinline__ void cfma(cpx<T>& acc, cpx<T> a, cpx<T> b) {
  acc.re = fma(a.re, b.re, acc.re);
  acc.re = fma(-a.im, b.im, acc.re);
  acc.im = fma(a.re, b.im, acc.im);
  acc.im = fma(a.im, b.re, acc.im);
}
template <typename T>
__device__ __forceinline__ void cfmac(cpx<T>& acc, cpx<T> a, cpx<T> b) {
  acc.re = fma(a.re, b.re, acc.re);
  acc.re = fma(a.im, b.im, acc.re);
  acc.im = fma(a.re, b.im, acc.im);
  acc.im = fma(-a.im, b.re, acc.im);
}
// i * a
template <typename T>
__host__ __device__ __forceinline__ cpx<T> mul_i(cpx<T> a) {
  return mk(-a.im, a.re);
}
template <typename T>
__host__ __device__ __forceinline__ T abs2(cpx<T> a) {
  return a.re * a.re + a.im * a.im;
}
template <typename TO, typename TI>
__host__ __device__ __forceinline__ cpx<TO> cvt(cpx<TI> a) {
  return mk(static_cast<TO>(a.re), static_cast<TO>(a.im));
}

using c64 = cpx<double>;  // complex128
using c32 = cpx<float>;   // complex64

// ----------------------------------------------------------------------------------------
// error plumbing: every C entry point returns a status; the message is kept per thread
// ----------------------------------------------------------------------------------------
void set_error(const std::string& msg);
const char* get_error();

#define KC_HIP(expr)                                                                  \
  do {                                                                                \
    hipError_t e_ = (expr);                                                           \
    if (e_ != hipSuccess) {                                                           \
      ::kc::set_error(std::string(#expr) + ": " + hipGetErrorString(e_));             \
      return KC_ERR_HIP;                                                              \
    }                                                                                 \
  } while (0)

#define KC_TRY(expr)            \
  do {                          \
    int s_ = (expr);            \
    if (s_ != KC_OK) return s_; \
  } while (0)

#define KC_ARG(cond, msg)                             \
  do {                                                \
    if (!(cond)) {                                    \
      ::kc::set_error(std::string("invalid argument: ") + (msg)); \
      return KC_ERR_INVALID_ARG;                      \
    }                                                 \
  } while (0)

// after a kernel launch
#define KC_LAUNCHED()                                                                  \
  do {                                                                                 \
    hipError_t e_ = hipGetLastError();                                                 \
    if (e_ != hipSuccess) {                                                            \
      ::kc::set_error(std::string("kernel launch: ") + hipGetErrorString(e_));         \
      return KC_ERR_HIP;                                                               \
    }                                                                                  \
  } while (0)

// Lattice transform of the difference symbols (Section 2.2, eq (2.12)): for primitive vectors
// other than the unit ones, K_i(p) = sum_j b_ji Lambda_1(q_j) + i k_i Lambda_0(q_i) with
// b = A^{-1}.  The per-axis tables hold K_i(q_i) = Lambda_1(q_i) + i k_i Lambda_0(q_i), so
// K_i(p) = K_i(q_i) + sum_j C_ij Lambda_1(q_j) with C_ij = b_ji - delta_ij.  l1d == nullptr
// means the simple-cubic lattice (C = 0).
struct Skew {
  const c32* l1f = nullptr;  // Lambda_1(q), q < N (complex64)
  const c64* l1d = nullptr;  // the same in complex128
  double c[9] = {0, 0, 0, 0, 0, 0, 0, 0, 0};
};

template <typename T>
__device__ __forceinline__ const cpx<T>* skew_l1(const Skew& s);
template <>
__device__ __forceinline__ const c32* skew_l1<float>(const Skew& s) {
  return s.l1f;
}
template <>
__device__ __forceinline__ const c64* skew_l1<double>(const Skew& s) {
  return s.l1d;
}

// K_1, K_2, K_3 of frequency (qx, qy, qz) from the per-axis values (no-op on the cubic lattice)
template <typename T>
__device__ __forceinline__ void skew_fix(const Skew& s, int qx, int qy, int qz, cpx<T>& K1, cpx<T>& K2,
                                         cpx<T>& K3) {
  if (s.l1d == nullptr) return;
  const cpx<T>* l = skew_l1<T>(s);
  const cpx<T> a = l[qx], b = l[qy], c = l[qz];
  K1 = K1 + static_cast<T>(s.c[0]) * a + static_cast<T>(s.c[1]) * b + static_cast<T>(s.c[2]) * c;
  K2 = K2 + static_cast<T>(s.c[3]) * a + static_cast<T>(s.c[4]) * b + static_cast<T>(s.c[5]) * c;
  K3 = K3 + static_cast<T>(s.c[6]) * a + static_cast<T>(s.c[7]) * b + static_cast<T>(s.c[8]) * c;
}

// Workgroup ids are dealt to the 8 XCDs of an MI355X round-robin (id % 8).  Remapping makes
// consecutive logical tiles land on the same XCD (and hence share its L2) while the grid is
// still spread evenly over the chip.  Requires nblocks to be a multiple of 8 to be a
// bijection; otherwise the identity is used.
__device__ __forceinline__ unsigned xcd_swizzle(unsigned b, unsigned nblocks) {
  if ((nblocks & 7u) != 0u) return b;
  const unsigned per = nblocks >> 3;
  return (b & 7u) * per + (b >> 3);
}

}  // namespace kc
