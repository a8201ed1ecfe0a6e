// Training support of the learned preconditioner (an addition to the paper's method, whose
// Section 4 solver uses the diagonal-block K_P^{-1} of eqs (2.31)-(2.32)): the exact
// corrections Op^{-1} r by preconditioned conjugate gradients, the residuals of perturbed
// eigenvector iterates that serve as training inputs, and the scale-free misfit of T_E r with
// its gradient with respect to the network output.  The operator, the preconditioners and the
// gradient of T_E run in the library's kernels; the per-vector inner products and
// combinations below are plain grid-stride kernels with fixed-order reductions.
#include <algorithm>
#include <cmath>
#include <vector>

#include "kc_nn.h"
#include "kc_state.h"

namespace kc {

namespace {

constexpr int TT = 256;      // threads per block
constexpr int TDOT = 240;    // blocks per vector (or pair) of an inner product

__device__ __forceinline__ double block_sum(double v, double* sh) {
  sh[threadIdx.x] = v;
  __syncthreads();
  for (int s = TT / 2; s > 0; s >>= 1) {
    if ((int)threadIdx.x < s) sh[threadIdx.x] += sh[threadIdx.x + s];
    __syncthreads();
  }
  return sh[0];
}

// part[j][blk] = partial sums of Re<a_j, b_j> = Re sum_t conj(a_j[t]) b_j[t]; grid (TDOT, nv)
__global__ __launch_bounds__(TT) void k_dot_part(const c64* __restrict__ a, const c64* __restrict__ b, size_t n,
                                                 double* __restrict__ part) {
  __shared__ double sh[TT];
  const size_t j = blockIdx.y;
  const c64* aj = a + j * n;
  const c64* bj = b + j * n;
  double acc = 0.0;
  for (size_t t = (size_t)blockIdx.x * TT + threadIdx.x; t < n; t += (size_t)gridDim.x * TT)
    acc += aj[t].re * bj[t].re + aj[t].im * bj[t].im;
  const double s = block_sum(acc, sh);
  if (threadIdx.x == 0) part[j * gridDim.x + blockIdx.x] = s;
}

// part[i][j][blk] = partial sums of the complex <a_i, b_j>; grid (TDOT, na * nb)
__global__ __launch_bounds__(TT) void k_cdot_part(const c64* __restrict__ a, const c64* __restrict__ b, size_t n,
                                                  int nb, double* __restrict__ part) {
  __shared__ double sh[TT];
  const int i = blockIdx.y / nb, j = blockIdx.y % nb;
  const c64* ai = a + (size_t)i * n;
  const c64* bj = b + (size_t)j * n;
  double re = 0.0, im = 0.0;
  for (size_t t = (size_t)blockIdx.x * TT + threadIdx.x; t < n; t += (size_t)gridDim.x * TT) {
    re += ai[t].re * bj[t].re + ai[t].im * bj[t].im;
    im += ai[t].re * bj[t].im - ai[t].im * bj[t].re;
  }
  const double sr = block_sum(re, sh);
  const double si = block_sum(im, sh);
  if (threadIdx.x == 0) {
    part[(2 * (size_t)blockIdx.y) * gridDim.x + blockIdx.x] = sr;
    part[(2 * (size_t)blockIdx.y + 1) * gridDim.x + blockIdx.x] = si;
  }
}

// out[j] = sum of part[j][0 .. nblk) in index order
__global__ void k_sum_parts(const double* __restrict__ part, int nblk, int nv, double* __restrict__ out) {
  const int j = blockIdx.x * blockDim.x + threadIdx.x;
  if (j >= nv) return;
  double s = 0.0;
  for (int t = 0; t < nblk; ++t) s += part[(size_t)j * nblk + t];
  out[j] = s;
}

// c_j += (rz_j / pAp_j) p_j,  res_j -= (rz_j / pAp_j) Ap_j  (a vector whose direction vanished,
// e.g. a zero right-hand side, stays where it is)
__global__ __launch_bounds__(TT) void k_cg_step(c64* __restrict__ c, c64* __restrict__ res, const c64* __restrict__ p,
                                                const c64* __restrict__ Ap, const double* __restrict__ rz,
                                                const double* __restrict__ pAp, size_t n) {
  const size_t j = blockIdx.y;
  const double al = pAp[j] > 0.0 ? rz[j] / pAp[j] : 0.0;
  for (size_t t = (size_t)blockIdx.x * TT + threadIdx.x; t < n; t += (size_t)gridDim.x * TT) {
    const size_t q = j * n + t;
    c[q] = c[q] + al * p[q];
    res[q] = res[q] - al * Ap[q];
  }
}

// p_j = z_j + (rz_new_j / rz_j) p_j
__global__ __launch_bounds__(TT) void k_cg_dir(c64* __restrict__ p, const c64* __restrict__ z,
                                               const double* __restrict__ rz_new, const double* __restrict__ rz,
                                               size_t n) {
  const size_t j = blockIdx.y;
  const double be = rz[j] != 0.0 ? rz_new[j] / rz[j] : 0.0;
  for (size_t t = (size_t)blockIdx.x * TT + threadIdx.x; t < n; t += (size_t)gridDim.x * TT) {
    const size_t q = j * n + t;
    p[q] = z[q] + be * p[q];
  }
}

// e_j -= sum_i G[i][j] X_i   (G[i][j] = <X_i, e_j>, complex, [m][m][2])
__global__ __launch_bounds__(TT) void k_project_out(c64* __restrict__ e, const c64* __restrict__ X,
                                                    const double* __restrict__ G, int m, size_t n) {
  const size_t j = blockIdx.y;
  for (size_t t = (size_t)blockIdx.x * TT + threadIdx.x; t < n; t += (size_t)gridDim.x * TT) {
    c64 v = e[j * n + t];
    for (int i = 0; i < m; ++i) {
      const c64 g = mk(G[2 * ((size_t)i * m + j)], G[2 * ((size_t)i * m + j) + 1]);
      v = v - g * X[(size_t)i * n + t];
    }
    e[j * n + t] = v;
  }
}

// x_j = X_j + (amp_j / |e_j|) e_j   (en2_j = |e_j|^2)
__global__ __launch_bounds__(TT) void k_perturb(c64* __restrict__ x, const c64* __restrict__ X,
                                                const c64* __restrict__ e, const double* __restrict__ amp,
                                                const double* __restrict__ en2, size_t n) {
  const size_t j = blockIdx.y;
  const double s = en2[j] > 0.0 ? amp[j] / sqrt(en2[j]) : 0.0;  // noise inside span(X): x = X
  for (size_t t = (size_t)blockIdx.x * TT + threadIdx.x; t < n; t += (size_t)gridDim.x * TT) {
    const size_t q = j * n + t;
    x[q] = X[q] + s * e[q];
  }
}

// y_j = a_j u_j - v_j
__global__ __launch_bounds__(TT) void k_scale_sub(c64* __restrict__ y, const c64* __restrict__ u,
                                                  const c64* __restrict__ v, const double* __restrict__ a,
                                                  size_t n) {
  const size_t j = blockIdx.y;
  const double s = a[j];
  for (size_t t = (size_t)blockIdx.x * TT + threadIdx.x; t < n; t += (size_t)gridDim.x * TT) {
    const size_t q = j * n + t;
    y[q] = s * u[q] - v[q];
  }
}

// r_j = Ax_j - (xAx_j / xx_j) x_j
__global__ __launch_bounds__(TT) void k_rayleigh_resid(c64* __restrict__ r, const c64* __restrict__ Ax,
                                                       const c64* __restrict__ x, const double* __restrict__ xAx,
                                                       const double* __restrict__ xx, size_t n) {
  const size_t j = blockIdx.y;
  const double th = xAx[j] / xx[j];
  for (size_t t = (size_t)blockIdx.x * TT + threadIdx.x; t < n; t += (size_t)gridDim.x * TT) {
    const size_t q = j * n + t;
    r[q] = Ax[q] - th * x[q];
  }
}

// gout[p][c] = scale * dL/dE_c(p) * E_c(p) where |y_c(p)| < 3 (E = E0 exp(clamp(y, -3, 3))),
// c < 3; the other channels of the 16-wide output are zero
__global__ __launch_bounds__(TT) void k_field_chain(float* __restrict__ gout, const float* __restrict__ gE,
                                                    const float* __restrict__ E, const float* __restrict__ y,
                                                    size_t N3, float scale) {
  for (size_t p = (size_t)blockIdx.x * TT + threadIdx.x; p < N3; p += (size_t)gridDim.x * TT) {
#pragma unroll
    for (int c = 0; c < 16; ++c) {
      float g = 0.f;
      if (c < 3 && fabsf(y[p * 16 + c]) < 3.f) g = scale * gE[c * N3 + p] * E[c * N3 + p];
      gout[p * 16 + c] = g;
    }
  }
}

unsigned grid_x(size_t n) { return (unsigned)std::min<size_t>((n + TT - 1) / TT, 1024); }

// Per-vector Re<a_j, b_j> of nv vectors of length n into out (device, nv doubles); part holds
// nv * TDOT doubles.
int dots(const c64* a, const c64* b, int nv, size_t n, double* part, double* out, hipStream_t s) {
  k_dot_part<<<dim3(TDOT, nv), TT, 0, s>>>(a, b, n, part);
  KC_LAUNCHED();
  k_sum_parts<<<(nv + 63) / 64, 64, 0, s>>>(part, TDOT, nv, out);
  KC_LAUNCHED();
  return KC_OK;
}

int to_host(std::vector<double>& h, const double* d, int nv, hipStream_t s) {
  h.resize(nv);
  KC_HIP(hipMemcpyAsync(h.data(), d, nv * sizeof(double), hipMemcpyDeviceToHost, s));
  KC_HIP(hipStreamSynchronize(s));
  return KC_OK;
}

int to_dev(double* d, const std::vector<double>& h, hipStream_t s) {
  KC_HIP(hipMemcpyAsync(d, h.data(), h.size() * sizeof(double), hipMemcpyHostToDevice, s));
  KC_HIP(hipStreamSynchronize(s));
  return KC_OK;
}

}  // namespace

}  // namespace kc

using namespace kc;

int kc_pcg(kc_op* op, int ik, int nvec, const void* r_, void* c_, double tol, int maxit, int* iters, void* stream) {
  KC_ARG(op != nullptr && op->nk > 0, "op with k-points");
  KC_ARG(ik >= 0 && ik < op->nk, "k-point index out of range");
  KC_ARG(nvec >= 1 && nvec <= 256, "1 <= nvec <= 256");
  KC_ARG(r_ != nullptr && c_ != nullptr, "NULL vector");
  KC_ARG(std::isfinite(tol) && tol > 0.0 && maxit >= 1, "tol > 0, maxit >= 1");
  const size_t n = 3 * (size_t)op->N * op->N * op->N;
  KC_ARG((const char*)c_ + nvec * n * sizeof(c64) <= (const char*)r_ ||
             (const char*)r_ + nvec * n * sizeof(c64) <= (const char*)c_,
         "r and c must not overlap");
  hipStream_t s = (hipStream_t)stream;
  const c64* r = (const c64*)r_;
  c64* c = (c64*)c_;
  const size_t vb = (size_t)nvec * n;
  KC_TRY(op->train_buf.ensure(4 * vb * sizeof(c64) + (size_t)nvec * (TDOT + 4) * sizeof(double)));
  c64* res = op->train_buf.as<c64>();
  c64* z = res + vb;
  c64* p = z + vb;
  c64* Ap = p + vb;
  double* part = reinterpret_cast<double*>(Ap + vb);
  double* rz = part + (size_t)nvec * TDOT;
  double* rz2 = rz + nvec;
  double* pAp = rz2 + nvec;
  double* rn = pAp + nvec;
  KC_TRY(build_efield(op));
  VecMap vm;
  vm.vpk = nvec;
  vm.kstride = nvec;
  const dim3 g(grid_x(n), nvec);
  KC_HIP(hipMemsetAsync(c, 0, vb * sizeof(c64), s));
  KC_HIP(hipMemcpyAsync(res, r, vb * sizeof(c64), hipMemcpyDeviceToDevice, s));
  KC_TRY(apply_tp(op, ik, nvec, vm, vm, res, z, op->efield.as<float>(), 0, KC_PREC_FP64, s));
  KC_HIP(hipMemcpyAsync(p, z, vb * sizeof(c64), hipMemcpyDeviceToDevice, s));
  KC_TRY(dots(res, z, nvec, n, part, rz, s));
  std::vector<double> r0, rh;
  KC_TRY(dots(r, r, nvec, n, part, rn, s));
  KC_TRY(to_host(r0, rn, nvec, s));
  int it = 0;
  bool conv = false;
  while (it < maxit && !conv) {
    KC_TRY(apply_op(op, ik, nvec, vm, p, Ap, KC_PREC_FP64, s));
    KC_TRY(dots(p, Ap, nvec, n, part, pAp, s));
    k_cg_step<<<g, TT, 0, s>>>(c, res, p, Ap, rz, pAp, n);
    KC_LAUNCHED();
    ++it;
    KC_TRY(dots(res, res, nvec, n, part, rn, s));
    KC_TRY(to_host(rh, rn, nvec, s));
    conv = true;
    for (int j = 0; j < nvec; ++j) conv = conv && (r0[j] == 0.0 || std::sqrt(rh[j]) <= tol * std::sqrt(r0[j]));
    if (conv) break;
    KC_TRY(apply_tp(op, ik, nvec, vm, vm, res, z, op->efield.as<float>(), 0, KC_PREC_FP64, s));
    KC_TRY(dots(res, z, nvec, n, part, rz2, s));
    k_cg_dir<<<g, TT, 0, s>>>(p, z, rz2, rz, n);
    KC_LAUNCHED();
    std::swap(rz, rz2);
  }
  KC_HIP(hipStreamSynchronize(s));
  if (iters) *iters = it;
  if (!conv) {
    set_error("kc_pcg: no convergence within maxit iterations");
    return KC_ERR_NO_CONVERGENCE;
  }
  return KC_OK;
}

int kc_perturbed_residuals(kc_op* op, int ik, int m, const void* X_, const void* noise_, const double* amp,
                           void* x_, void* r_, void* stream) {
  KC_ARG(op != nullptr && op->nk > 0, "op with k-points");
  KC_ARG(ik >= 0 && ik < op->nk, "k-point index out of range");
  KC_ARG(m >= 1 && m <= 32, "1 <= m <= 32");
  KC_ARG(X_ != nullptr && noise_ != nullptr && amp != nullptr && r_ != nullptr, "NULL argument");
  for (int j = 0; j < m; ++j) KC_ARG(std::isfinite(amp[j]), "amp must be finite");
  const size_t n = 3 * (size_t)op->N * op->N * op->N;
  hipStream_t s = (hipStream_t)stream;
  const c64* X = (const c64*)X_;
  c64* r = (c64*)r_;
  const size_t vb = (size_t)m * n;
  KC_TRY(op->train_buf.ensure(3 * vb * sizeof(c64) + ((size_t)2 * m * m * TDOT + 2 * m * m + 5 * m) * sizeof(double)));
  c64* e = op->train_buf.as<c64>();
  c64* x = e + vb;
  c64* Ax = x + vb;
  double* part = reinterpret_cast<double*>(Ax + vb);
  double* G = part + (size_t)2 * m * m * TDOT;
  double* en2 = G + 2 * m * m;
  double* ampd = en2 + m;
  double* xAx = ampd + m;
  double* xx = xAx + m;
  const dim3 g(grid_x(n), m);
  VecMap vm;
  vm.vpk = m;
  vm.kstride = m;
  // e = K_P^{-1} noise, then the orthogonal projection onto span(X) taken away
  KC_TRY(apply_precond(op, ik, m, m, (const c64*)noise_, e, s));
  k_cdot_part<<<dim3(TDOT, m * m), TT, 0, s>>>(X, e, n, m, part);
  KC_LAUNCHED();
  k_sum_parts<<<(2 * m * m + 63) / 64, 64, 0, s>>>(part, TDOT, 2 * m * m, G);
  KC_LAUNCHED();
  k_project_out<<<g, TT, 0, s>>>(e, X, G, m, n);
  KC_LAUNCHED();
  KC_TRY(dots(e, e, m, n, part, en2, s));
  std::vector<double> ah(amp, amp + m);
  KC_TRY(to_dev(ampd, ah, s));
  k_perturb<<<g, TT, 0, s>>>(x, X, e, ampd, en2, n);
  KC_LAUNCHED();
  KC_TRY(apply_op(op, ik, m, vm, x, Ax, KC_PREC_FP64, s));
  KC_TRY(dots(x, Ax, m, n, part, xAx, s));
  KC_TRY(dots(x, x, m, n, part, xx, s));
  k_rayleigh_resid<<<g, TT, 0, s>>>(r, Ax, x, xAx, xx, n);
  KC_LAUNCHED();
  if (x_ != nullptr) KC_HIP(hipMemcpyAsync(x_, x, vb * sizeof(c64), hipMemcpyDeviceToDevice, s));
  KC_HIP(hipStreamSynchronize(s));
  return KC_OK;
}

int kc_net_loss_grad(kc_op* op, int ik, int nvec, const void* r_, const void* c_, int kind, double scale, double* loss,
                     float* gout, void* stream) {
  KC_ARG(op != nullptr && op->nk > 0 && op->net != nullptr, "op with k-points and an attached network");
  KC_ARG(ik >= 0 && ik < op->nk, "k-point index out of range");
  KC_ARG(nvec >= 1 && nvec <= 256, "1 <= nvec <= 256");
  KC_ARG(r_ != nullptr && c_ != nullptr && loss != nullptr, "NULL argument");
  KC_ARG(kind == 0 || kind == 1, "kind: 0 (energy) or 1 (Euclidean)");
  KC_ARG(std::isfinite(scale), "scale must be finite");
  const size_t N3 = (size_t)op->N * op->N * op->N;
  const size_t n = 3 * N3;
  hipStream_t s = (hipStream_t)stream;
  const c64* r = (const c64*)r_;
  const c64* c = (const c64*)c_;
  const size_t vb = (size_t)nvec * n;
  KC_TRY(op->train_buf.ensure(3 * vb * sizeof(c64) + (size_t)nvec * (TDOT + 6) * sizeof(double) +
                              3 * N3 * sizeof(float)));
  c64* z = op->train_buf.as<c64>();
  c64* Oz = z + vb;
  c64* ge = Oz + vb;
  double* part = reinterpret_cast<double*>(ge + vb);
  double* d0 = part + (size_t)nvec * TDOT;
  double* d1 = d0 + nvec;
  double* d2 = d1 + nvec;
  double* al = d2 + nvec;
  double* w = al + nvec;
  double* d3 = w + nvec;
  float* gE = reinterpret_cast<float*>(d3 + nvec);
  const dim3 g(grid_x(n), nvec);
  VecMap vm;
  vm.vpk = nvec;
  vm.kstride = nvec;
  // the network's field for this k-point (its output y stays in the network's buffer)
  KC_TRY(learned_fields(op, ik, 1, s));
  const float* E = op->efield_k.as<float>();
  KC_TRY(apply_tp(op, ik, nvec, vm, vm, r, z, E, 1, KC_PREC_FP64, s));
  std::vector<double> h0, h1, h2, ha(nvec), hw(nvec);
  double sum = 0.0;
  if (kind == 0) {
    // 1 - (z^H r)^2 / ((z^H Op z)(c^H r)); alpha = z^H r / z^H Op z; Op e = alpha Op z - r
    KC_TRY(apply_op(op, ik, nvec, vm, z, Oz, KC_PREC_FP64, s));
    KC_TRY(dots(c, r, nvec, n, part, d0, s));
    KC_TRY(dots(z, r, nvec, n, part, d1, s));
    KC_TRY(dots(z, Oz, nvec, n, part, d2, s));
    KC_TRY(to_host(h0, d0, nvec, s));
    KC_TRY(to_host(h1, d1, nvec, s));
    KC_TRY(to_host(h2, d2, nvec, s));
    for (int j = 0; j < nvec; ++j) {
      if (!(h0[j] > 0.0 && h2[j] > 0.0)) {
        set_error("kc_net_loss_grad: a residual or its preconditioned direction has no energy");
        return KC_ERR_INVALID_ARG;
      }
      sum += 1.0 - h1[j] * h1[j] / (h2[j] * h0[j]);
      ha[j] = h1[j] / h2[j];
      hw[j] = 2.0 * ha[j] / (h0[j] * nvec);
    }
    *loss = sum / nvec;
    if (gout == nullptr) return KC_OK;
    KC_TRY(to_dev(al, ha, s));
    k_scale_sub<<<g, TT, 0, s>>>(ge, Oz, r, al, n);
    KC_LAUNCHED();
  } else {
    // min_alpha |alpha z - c|^2 / |c|^2, alpha = z^H c / z^H z, e = alpha z - c
    KC_TRY(dots(c, c, nvec, n, part, d0, s));
    KC_TRY(dots(z, c, nvec, n, part, d1, s));
    KC_TRY(dots(z, z, nvec, n, part, d2, s));
    KC_TRY(to_host(h0, d0, nvec, s));
    KC_TRY(to_host(h1, d1, nvec, s));
    KC_TRY(to_host(h2, d2, nvec, s));
    for (int j = 0; j < nvec; ++j) {
      if (!(h0[j] > 0.0 && h2[j] > 0.0)) {
        set_error("kc_net_loss_grad: a target or a preconditioned residual is zero");
        return KC_ERR_INVALID_ARG;
      }
      ha[j] = h1[j] / h2[j];
      hw[j] = 2.0 * ha[j] / (h0[j] * nvec);
    }
    KC_TRY(to_dev(al, ha, s));
    k_scale_sub<<<g, TT, 0, s>>>(ge, z, c, al, n);
    KC_LAUNCHED();
    std::vector<double> h3;
    KC_TRY(dots(ge, ge, nvec, n, part, d3, s));
    KC_TRY(to_host(h3, d3, nvec, s));
    for (int j = 0; j < nvec; ++j) sum += h3[j] / h0[j];
    *loss = sum / nvec;
    if (gout == nullptr) return KC_OK;
  }
  // dL/dE = sum_j w_j Re(conj(G Op e_j) G r_j) (energy) or with e_j itself (Euclidean), G = F3 K_A^+
  KC_TRY(to_dev(w, hw, s));
  KC_HIP(hipMemsetAsync(gE, 0, 3 * N3 * sizeof(float), s));
  KC_TRY(tp_grad(op, ik, nvec, nvec, r, ge, w, gE, s));
  k_field_chain<<<grid_x(N3), TT, 0, s>>>(gout, gE, E, op->net->out.as<float>(), N3, (float)scale);
  KC_LAUNCHED();
  KC_HIP(hipStreamSynchronize(s));
  return KC_OK;
}
