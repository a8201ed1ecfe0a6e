// C ABI entry points (include/kcpc.h): argument checking, set-up of the per-k symbol tables,
// the inverse-permittivity table and the twiddles, and dispatch to the kernels.
#include <algorithm>
#include <cmath>
#include <complex>
#include <cstring>
#include <map>
#include <mutex>
#include <string>

#include "kc_blas.h"
#include "kc_nn.h"

namespace kc {

static thread_local std::string g_err;
void set_error(const std::string& msg) { g_err = msg; }
const char* get_error() { return g_err.c_str(); }

int DevBuf::ensure(size_t n) {
  if (n <= bytes && p != nullptr) return KC_OK;
  release();
  if (n == 0) return KC_OK;
  if (al != nullptr && al->alloc != nullptr) {
    p = al->alloc(al->ctx, n);
    if (p == nullptr) {
      set_error("caller allocator returned NULL for " + std::to_string(n) + " bytes");
      return KC_ERR_ALLOC;
    }
    // the caller's memory may have been in use on another stream until now
    KC_HIP(hipDeviceSynchronize());
  } else {
    hipError_t e = hipMalloc(&p, n);
    if (e != hipSuccess) {
      p = nullptr;
      set_error(std::string("hipMalloc(") + std::to_string(n) + "): " + hipGetErrorString(e));
      return KC_ERR_ALLOC;
    }
  }
  bytes = n;
  hipError_t e = hipMemset(p, 0, n);
  if (e != hipSuccess) {
    set_error(std::string("hipMemset: ") + hipGetErrorString(e));
    return KC_ERR_HIP;
  }
  return KC_OK;
}

void DevBuf::release() {
  if (p) {
    if (al != nullptr && al->free != nullptr)
      al->free(al->ctx, p, bytes);
    else
      (void)hipFree(p);
  }
  p = nullptr;
  bytes = 0;
}

int fft3d(int N, int nvec, int sign, int prec, const void* in, void* out, const void* tw, hipStream_t s);
void solver_release(kc_op* op);

static bool supported_n(int N) {
  switch (N) {
    case 4: case 6: case 8: case 12: case 16: case 24: case 32: case 48: case 64: case 96: case 128:
      return true;
    default:
      return false;
  }
}

// twiddles exp(+2 pi i t/N), t < N, from long double
static void make_twiddles(int N, std::vector<c64>& d, std::vector<c32>& f) {
  d.resize(N);
  f.resize(N);
  const long double pi = 3.141592653589793238462643383279502884L;
  for (int t = 0; t < N; ++t) {
    const long double a = 2.0L * pi * (long double)t / (long double)N;
    const long double c = std::cos(a), s = std::sin(a);
    d[t] = mk((double)c, (double)s);
    f[t] = mk((float)c, (float)s);
  }
}

template <typename T>
static int upload(DevBuf& b, const std::vector<T>& v, hipStream_t s = nullptr) {
  KC_TRY(b.ensure(v.size() * sizeof(T)));
  KC_HIP(hipMemcpyAsync(b.p, v.data(), v.size() * sizeof(T), hipMemcpyHostToDevice, s));
  KC_HIP(hipStreamSynchronize(s));
  return KC_OK;
}

// Coefficients c_s^(1), c_s^(0) (s = 1..m) of the order-2m stencils of eq (2.34): the m x m
// system of eq (2.35), sum_t ((2t - 1)/2)^(2s + kind - 2) c_t = 1/2 for s = 1 and 0 for s > 1,
// solved by Gaussian elimination with partial pivoting in long double (the solution is a set of
// small dyadic-like rationals, Table 1; the result is exact to double rounding).
static void stencil_coeffs(int m, double c1[5], double c0[5]) {
  for (int kind = 1; kind >= 0; --kind) {
    long double A[5][6] = {};
    for (int s = 1; s <= m; ++s) {
      for (int t = 1; t <= m; ++t) {
        const long double b = (2.0L * t - 1.0L) / 2.0L;
        long double pw = 1.0L;
        for (int e = 0; e < 2 * s + kind - 2; ++e) pw *= b;
        A[s - 1][t - 1] = pw;
      }
      A[s - 1][m] = (s == 1) ? 0.5L : 0.0L;
    }
    for (int c = 0; c < m; ++c) {
      int piv = c;
      for (int r = c + 1; r < m; ++r)
        if (std::fabs((double)A[r][c]) > std::fabs((double)A[piv][c])) piv = r;
      for (int j = 0; j <= m; ++j) std::swap(A[c][j], A[piv][j]);
      for (int r = 0; r < m; ++r) {
        if (r == c) continue;
        const long double f = A[r][c] / A[c][c];
        for (int j = c; j <= m; ++j) A[r][j] -= f * A[c][j];
      }
    }
    for (int s = 0; s < 5; ++s) (kind ? c1 : c0)[s] = s < m ? (double)(A[s][m] / A[s][s]) : 0.0;
  }
}

// Gershgorin test of the discrete inverse permittivity M: every row's diagonal entry exceeds the
// sum of the moduli of its off-diagonal entries (then the Hermitian M is positive definite).
// Trivial (eq (3.4)): row c of cell p couples to the two other components of the same cell
// through the volume-point entries.  CrossDoF (eq (3.8) with the entries sampled per point set):
// the (c, d) block is (Q_c T + T Q_d) / 2 with four transfer weights 1/4, so an entry between
// a c-edge P and a d-edge S is (eps_cd(P) + eps_cd(S)) / 8; for c > d the conjugate transpose.
static bool gershgorin_hpd(int N, int scheme, const uint8_t* ids, const double* tab) {
  if (scheme == KC_EPS_DIAGONAL) return true;  // diagonal entries are positive (Assumption 3.1)
  const size_t N3 = (size_t)N * N * N;
  auto ent = [&](int mat, int r, int c) {
    const double* t = tab + ((size_t)mat * 9 + r * 3 + c) * 2;
    return std::hypot(t[0], t[1]);
  };
  auto idx = [&](int i, int j, int k) {
    return (size_t)((i % N + N) % N) + (size_t)N * ((j % N + N) % N) + (size_t)N * N * ((k % N + N) % N);
  };
  for (int k = 0; k < N; ++k)
    for (int j = 0; j < N; ++j)
      for (int i = 0; i < N; ++i) {
        const size_t p = idx(i, j, k);
        for (int c = 0; c < 3; ++c) {
          const double d = tab[((size_t)ids[c * N3 + p] * 9 + c * 4) * 2];
          double off = 0.0;
          if (scheme == KC_EPS_TRIVIAL) {
            for (int e = 0; e < 3; ++e)
              if (e != c) off += ent(ids[3 * N3 + p], c, e);
          } else {
            // the four e-edges nearest to the c-edge of cell p (the transfer stencils of
            // eqs (3.5)-(3.7) read geometrically, and their transposes): cell offsets {0, -1}
            // along the c axis and {0, +1} along the e axis, for c < e and for c > e alike
            for (int e = 0; e < 3; ++e) {
              if (e == c) continue;
              const double ep = ent(ids[c * N3 + p], c, e);
              for (int a = 0; a < 2; ++a)
                for (int b = 0; b < 2; ++b) {
                  int o[3] = {0, 0, 0};
                  o[c] = -a;
                  o[e] = b;
                  const size_t q = idx(i + o[0], j + o[1], k + o[2]);
                  off += 0.125 * (ep + ent(ids[e * N3 + q], c, e));
                }
            }
          }
          if (!(d > off)) return false;
        }
      }
  return true;
}

// Hermitian 3x3 check of Assumption 3.1 (eigenvalues in (0, 1]): Cholesky of A (positive
// definite) and of I - A + tol I (I - A positive semi-definite).
static bool chol3_pd(std::complex<double> A[3][3]) {
  std::complex<double> L[3][3] = {};
  for (int j = 0; j < 3; ++j) {
    double d = A[j][j].real();
    for (int k = 0; k < j; ++k) d -= std::norm(L[j][k]);
    if (!(d > 0.0)) return false;
    L[j][j] = std::sqrt(d);
    for (int i = j + 1; i < 3; ++i) {
      std::complex<double> s = A[i][j];
      for (int k = 0; k < j; ++k) s -= L[i][k] * std::conj(L[j][k]);
      L[i][j] = s / L[j][j].real();
    }
  }
  return true;
}

static int check_table(int n_mat, const double* t) {
  for (int m = 0; m < n_mat; ++m) {
    std::complex<double> A[3][3], B[3][3];
    for (int r = 0; r < 3; ++r)
      for (int c = 0; c < 3; ++c) A[r][c] = {t[((m * 3 + r) * 3 + c) * 2], t[((m * 3 + r) * 3 + c) * 2 + 1]};
    double scale = 0.0;
    for (int r = 0; r < 3; ++r)
      for (int c = 0; c < 3; ++c) scale = std::max(scale, std::abs(A[r][c]));
    for (int r = 0; r < 3; ++r)
      for (int c = 0; c < 3; ++c)
        if (std::abs(A[r][c] - std::conj(A[c][r])) > 1e-12 * std::max(scale, 1.0)) {
          set_error("inverse permittivity of material " + std::to_string(m) + " is not Hermitian");
          return KC_ERR_NOT_HPD;
        }
    for (int r = 0; r < 3; ++r)
      for (int c = 0; c < 3; ++c) B[r][c] = (r == c ? 1.0 + 1e-12 : 0.0) - A[r][c];
    if (!chol3_pd(A) || !chol3_pd(B)) {
      set_error("inverse permittivity of material " + std::to_string(m) +
                " has an eigenvalue outside (0, 1] (Assumption 3.1)");
      return KC_ERR_NOT_HPD;
    }
  }
  return KC_OK;
}

// v *= a over a flat array (grid-stride)
__global__ void k_scale(c64* v, size_t n, double a) {
  for (size_t i = blockIdx.x * (size_t)blockDim.x + threadIdx.x; i < n; i += (size_t)gridDim.x * blockDim.x)
    v[i] = a * v[i];
}

// per-N twiddle tables for kc_fft3d (one set per process and device)
struct TwCache {
  std::mutex mu;
  std::map<std::pair<int, int>, DevBuf*> tabs;  // (device, N) -> [c64 N | c32 N]
};
static TwCache& twcache() {
  static TwCache* c = new TwCache();  // never destroyed: outlives static destructors
  return *c;
}

}  // namespace kc

using namespace kc;

extern "C" {

int kc_supported_n(int N) { return supported_n(N) ? 1 : 0; }

int kc_create(int N, const double* lattice_host, int stencil_m, int eps_scheme, const uint8_t* mat_ids_host,
              int n_mat, const double* eps_inv_host, kc_alloc_fn alloc, kc_free_fn free_fn, void* alloc_ctx,
              void* stream, kc_op** out) {
  KC_ARG(out != nullptr, "out is NULL");
  *out = nullptr;
  if (!supported_n(N)) {
    set_error("grid division N=" + std::to_string(N) + " is not a supported FFT length");
    return KC_ERR_UNSUPPORTED;
  }
  // lattice: A = (a_1 a_2 a_3) with the primitive vectors as columns, b = A^{-1} (Section 2.2);
  // the symbols need C_ij = b_ji - delta_ij (eq (2.12))
  double cmat[9] = {0, 0, 0, 0, 0, 0, 0, 0, 0};
  bool skewed = false;
  if (lattice_host != nullptr) {
    double A[3][3];
    for (int r = 0; r < 3; ++r)
      for (int c = 0; c < 3; ++c) {
        KC_ARG(std::isfinite(lattice_host[r * 3 + c]), "non-finite lattice vector");
        A[c][r] = lattice_host[r * 3 + c];  // vector r is column r of A
      }
    const double det = A[0][0] * (A[1][1] * A[2][2] - A[1][2] * A[2][1]) -
                       A[0][1] * (A[1][0] * A[2][2] - A[1][2] * A[2][0]) +
                       A[0][2] * (A[1][0] * A[2][1] - A[1][1] * A[2][0]);
    double nrm = 0.0;
    for (int r = 0; r < 3; ++r)
      for (int c = 0; c < 3; ++c) nrm = std::max(nrm, std::fabs(A[r][c]));
    KC_ARG(std::fabs(det) > 1e-9 * nrm * nrm * nrm, "lattice vectors are linearly dependent");
    double b[3][3];  // inverse by cofactors
    for (int r = 0; r < 3; ++r)
      for (int c = 0; c < 3; ++c) {
        const int r1 = (c + 1) % 3, r2 = (c + 2) % 3, c1 = (r + 1) % 3, c2 = (r + 2) % 3;
        b[r][c] = (A[r1][c1] * A[r2][c2] - A[r1][c2] * A[r2][c1]) / det;
      }
    for (int i = 0; i < 3; ++i)
      for (int j = 0; j < 3; ++j) {
        cmat[i * 3 + j] = b[j][i] - (i == j ? 1.0 : 0.0);
        if (std::fabs(cmat[i * 3 + j]) > 1e-15) skewed = true;
      }
  }
  KC_ARG(stencil_m >= 1 && stencil_m <= 5, "stencil_m must be in [1, 5] (orders 2 to 10)");
  KC_ARG((alloc == nullptr) == (free_fn == nullptr), "alloc and free_fn must be given together");
  KC_ARG(eps_scheme == KC_EPS_DIAGONAL || eps_scheme == KC_EPS_TRIVIAL || eps_scheme == KC_EPS_CROSSDOF,
         "eps_scheme");
  KC_ARG(mat_ids_host != nullptr && eps_inv_host != nullptr, "NULL ids or table");
  KC_ARG(n_mat >= 1 && n_mat <= KC_MAX_MAT, "n_mat must be in [1, 64]");
  KC_TRY(check_table(n_mat, eps_inv_host));
  hipStream_t hs = (hipStream_t)stream;
  const size_t N3 = (size_t)N * N * N;
  std::vector<uint32_t> packed(N3);
  std::vector<char> present(n_mat, 0);
  for (size_t p = 0; p < N3; ++p) {
    uint32_t w = 0;
    for (int s = 0; s < 4; ++s) {
      const uint8_t id = mat_ids_host[s * N3 + p];
      if (id >= n_mat) {
        set_error("material id " + std::to_string(id) + " >= n_mat");
        return KC_ERR_INVALID_ARG;
      }
      present[id] = 1;
      w |= (uint32_t)id << (8 * s);
    }
    packed[p] = w;
  }
  kc_op* op = new kc_op();
  op->N = N;
  op->scheme = eps_scheme;
  op->n_mat = n_mat;
  op->stencil_m = stencil_m;
  op->alloc.alloc = alloc;
  op->alloc.free = free_fn;
  op->alloc.ctx = alloc_ctx;
  op->bind_allocator();
  if (!gershgorin_hpd(N, eps_scheme, mat_ids_host, eps_inv_host)) op->flags |= KC_FLAG_HPD_UNPROVEN;
  op->eps_host.assign(eps_inv_host, eps_inv_host + (size_t)n_mat * 18);
  op->epsinv_norm = 0.0;  // bounds |eps^-1| where the grid uses it (the scale of FP32 rounding)
  for (int m = 0; m < n_mat; ++m)
    if (present[m])
      for (int i = 0; i < 3; ++i) {
        double r = 0.0;
        for (int j = 0; j < 3; ++j) {
          const double* e = eps_inv_host + m * 18 + (i * 3 + j) * 2;
          r += std::hypot(e[0], e[1]);
        }
        op->epsinv_norm = std::max(op->epsinv_norm, r);
      }
  // permittivity entries scaled by 1/N^3 (normalisation of the two unnormalised DFTs)
  const double sc = 1.0 / (double)N3;
  std::vector<EpsEntry<double>> e64(n_mat);
  std::vector<EpsEntry<float>> e32(n_mat);
  const int offd[3][2] = {{0, 1}, {0, 2}, {1, 2}};
  for (int m = 0; m < n_mat; ++m) {
    const double* t = eps_inv_host + (size_t)m * 18;
    for (int c = 0; c < 3; ++c) {
      e64[m].d[c] = t[(c * 3 + c) * 2] * sc;
      e32[m].d[c] = (float)e64[m].d[c];
    }
    for (int q = 0; q < 3; ++q) {
      const int r = offd[q][0], c = offd[q][1];
      double re = t[(r * 3 + c) * 2] * sc, im = t[(r * 3 + c) * 2 + 1] * sc;
      if (eps_scheme == KC_EPS_DIAGONAL) re = im = 0.0;
      e64[m].o[q] = mk(re, im);
      e32[m].o[q] = mk((float)re, (float)im);
    }
  }
  op->zoff = false;
  for (int m = 0; m < n_mat; ++m)
    for (int q = 1; q < 3; ++q) op->zoff = op->zoff || e64[m].o[q].re != 0.0 || e64[m].o[q].im != 0.0;
  int st = upload(op->ids, packed, hs);
  if (st == KC_OK) st = upload(op->eps64, e64, hs);
  if (st == KC_OK) st = upload(op->eps32, e32, hs);
  std::vector<c64> twd;
  std::vector<c32> twf;
  make_twiddles(N, twd, twf);
  if (st == KC_OK) st = upload(op->tw64, twd, hs);
  if (st == KC_OK) st = upload(op->tw32, twf, hs);
  if (st == KC_OK && skewed) {
    // Lambda_1(q) = (1/h) sum_s c1_s (e^{i(s-1)theta} - e^{-i s theta}), theta = 2 pi q/N
    double c1[5], c0[5];
    stencil_coeffs(stencil_m, c1, c0);
    std::vector<c64> l64(N);
    std::vector<c32> l32(N);
    for (int q = 0; q < N; ++q) {
      const double th = 2.0 * M_PI * (double)q / (double)N;
      std::complex<double> l(0.0, 0.0);
      for (int t = 1; t <= stencil_m; ++t) l += c1[t - 1] * (std::polar(1.0, (t - 1) * th) - std::polar(1.0, -t * th));
      l *= (double)N;
      l64[q] = mk(l.real(), l.imag());
      l32[q] = mk((float)l.real(), (float)l.imag());
    }
    st = op->lam1.ensure(N * (sizeof(c64) + sizeof(c32)));
    if (st == KC_OK) {
      hipError_t e = hipMemcpyAsync(op->lam1.p, l64.data(), N * sizeof(c64), hipMemcpyHostToDevice, hs);
      if (e == hipSuccess)
        e = hipMemcpyAsync((char*)op->lam1.p + N * sizeof(c64), l32.data(), N * sizeof(c32), hipMemcpyHostToDevice,
                           hs);
      if (e == hipSuccess) e = hipStreamSynchronize(hs);
      if (e != hipSuccess) {
        set_error(std::string("upload of the lattice symbols: ") + hipGetErrorString(e));
        st = KC_ERR_HIP;
      }
    }
    op->lam1_host = l64;
    op->skew.l1d = op->lam1.as<c64>();
    op->skew.l1f = (const c32*)((const char*)op->lam1.p + N * sizeof(c64));
    for (int i = 0; i < 9; ++i) op->skew.c[i] = cmat[i];
  }
  if (st == KC_OK) st = prepare_kernels(N);
  if (st != KC_OK) {
    delete op;
    return st;
  }
  *out = op;
  return KC_OK;
}

int kc_set_kpoints(kc_op* op, int nk, const double* k_host, const double* gamma_host) {
  KC_ARG(op != nullptr, "op is NULL");
  KC_ARG(nk >= 1 && k_host != nullptr, "nk >= 1 and k_host required");
  const int N = op->N;
  const double h = 1.0 / N;
  const double fourpi2 = 4.0 * M_PI * M_PI;
  // every argument is checked before the handle changes
  std::vector<double> gam(nk);
  std::vector<int> kfl(nk, 0);
  for (int ik = 0; ik < nk; ++ik) {
    const double* k = k_host + 3 * ik;
    for (int a = 0; a < 3; ++a) {
      KC_ARG(std::isfinite(k[a]), "non-finite wave vector");
      if (std::fabs(k[a]) > M_PI) kfl[ik] |= KC_KFLAG_K_OUTSIDE;
    }
    const double kn2 = k[0] * k[0] + k[1] * k[1] + k[2] * k[2];
    double g;
    if (gamma_host) {
      g = gamma_host[ik];
      KC_ARG(std::isfinite(g) && g > 0.0, "gamma must be positive");
    } else {
      // Remark 2.6, eq (2.26)
      g = (kn2 == 0.0 || kn2 >= 1.0) ? fourpi2 : fourpi2 / kn2;
    }
    gam[ik] = g;
  }
  double c1[5], c0[5];
  stencil_coeffs(op->stencil_m, c1, c0);
  std::vector<c64> kt((size_t)nk * 3 * N);
  std::vector<c32> kf(kt.size());
  std::vector<double> smin(nk), smax(nk);
  std::vector<int> dcl(nk, 0);
  for (int ik = 0; ik < nk; ++ik) {
    const double* k = k_host + 3 * ik;
    double lo0[3], lo1[3], hi[3];  // smallest, second smallest and largest |K_a(q)|^2 over q
    for (int a = 0; a < 3; ++a) {
      lo0[a] = lo1[a] = INFINITY;
      hi[a] = 0.0;
      for (int q = 0; q < N; ++q) {
        // eigenvalues of the circulants D1 and D0 (first rows from eq (2.34)) by Lemma 2.1,
        // theta = 2 pi q/N: D1 -> (1/h) sum_s c1_s (e^{i(s-1)theta} - e^{-i s theta}),
        // D0 -> sum_s c0_s (e^{i(s-1)theta} + e^{-i s theta}); m = 1 gives (1 - e^{-i theta})/h
        // and (1 + e^{-i theta})/2 of eq (2.5).  K_a = D1 + i k_a D0 (eq (2.6)).
        const double th = 2.0 * M_PI * (double)q / (double)N;
        std::complex<double> l1(0.0, 0.0), l0(0.0, 0.0);
        for (int s = 1; s <= op->stencil_m; ++s) {
          const std::complex<double> ep = std::polar(1.0, (s - 1) * th), em = std::polar(1.0, -s * th);
          l1 += c1[s - 1] * (ep - em);
          l0 += c0[s - 1] * (ep + em);
        }
        l1 /= h;
        const std::complex<double> K = l1 + std::complex<double>(0.0, k[a]) * l0;
        kt[((size_t)ik * 3 + a) * N + q] = mk(K.real(), K.imag());
        kf[((size_t)ik * 3 + a) * N + q] = mk((float)K.real(), (float)K.imag());
        const double v = std::norm(K);
        hi[a] = std::max(hi[a], v);
        if (v < lo0[a]) {
          lo1[a] = lo0[a];
          lo0[a] = v;
        } else if (v < lo1[a]) {
          lo1[a] = v;
        }
      }
    }
    // smallest s(p) = sum_a |K_a(p)|^2 (s0) and the next value over the other frequencies (s2):
    // on the cubic lattice s is a sum of per-axis terms (all axes at their minimum; then one axis
    // at its second smallest), otherwise every frequency is visited
    double s0 = lo0[0] + lo0[1] + lo0[2];
    double s2 = INFINITY;
    for (int a = 0; a < 3; ++a) s2 = std::min(s2, s0 - lo0[a] + lo1[a]);
    double smx = hi[0] + hi[1] + hi[2];
    if (op->skew.l1d != nullptr) {
      const double* C = op->skew.c;
      std::vector<std::complex<double>> l1(N);
      for (int q = 0; q < N; ++q) {
        const double th = 2.0 * M_PI * (double)q / (double)N;
        std::complex<double> l(0.0, 0.0);
        for (int t = 1; t <= op->stencil_m; ++t)
          l += c1[t - 1] * (std::polar(1.0, (t - 1) * th) - std::polar(1.0, -t * th));
        l1[q] = l / h;
      }
      s0 = s2 = INFINITY;
      for (int qz = 0; qz < N; ++qz)
        for (int qy = 0; qy < N; ++qy)
          for (int qx = 0; qx < N; ++qx) {
            const int qq[3] = {qx, qy, qz};
            double sp = 0.0;
            for (int i = 0; i < 3; ++i) {
              const c64 t = kt[((size_t)ik * 3 + i) * N + qq[i]];
              std::complex<double> Ki(t.re, t.im);
              for (int j = 0; j < 3; ++j) Ki += C[i * 3 + j] * l1[qq[j]];
              sp += std::norm(Ki);
            }
            if (qx == 0 && qy == 0 && qz == 0) smx = 0.0;
            smx = std::max(smx, sp);
            if (sp < s0) {
              s2 = s0;
              s0 = sp;
            } else if (sp < s2) {
              s2 = sp;
            }
          }
    }
    smin[ik] = (s0 > 1e-300) ? s0 : s2;
    // Near Gamma (0 < |k| < 0.1) the rule of eq (2.26) gives gamma > 3948, growing as |k|^-2,
    // and the penalty block then dominates the Rayleigh-Ritz pencil in FP64.  There the solver
    // deflates the DC longitudinal direction instead (the constant field along k, an exact
    // eigenvector with eigenvalue gamma |k|^2, Prop 2.3) and gamma = 4 pi^2 / s2 keeps every
    // remaining penalty eigenvalue at or above 4 pi^2, the level the rule aims at.  Not applied
    // to a gamma the caller gives.
    smax[ik] = smx;
    const double kn2 = k[0] * k[0] + k[1] * k[1] + k[2] * k[2];
    if (!gamma_host && kn2 > 0.0 && kn2 < 0.01) {
      dcl[ik] = 1;
      gam[ik] = fourpi2 / s2;
      smin[ik] = s2;
    }
  }
  // no k-points while the tables change (a failed upload leaves none), then the sizes that the
  // range checks of the other calls read
  op->nk = 0;
  KC_TRY(upload(op->kdev, std::vector<double>(k_host, k_host + 3 * (size_t)nk)));
  KC_TRY(upload(op->ktab64, kt));
  KC_TRY(upload(op->ktab32, kf));
  op->ktab_host = kt;
  KC_TRY(upload(op->gamma_d, gam));
  // The solver's preconditioners (K_P^{-1}, T_E) take s = |K(p)|^2 no smaller than this floor:
  // near k = 0 the DC frequency has s = |k|^2 and a gain 1/|k|^2 that makes every new search
  // direction nearly the same constant field, so the Rayleigh-Ritz pencil loses its rank.  The
  // floor (1e-3 of (2 pi)^2, the size of s at the next frequencies) only changes the
  // preconditioner, not the operator or its eigenpairs.
  KC_TRY(upload(op->sfloor_d, std::vector<double>(nk, 4e-3 * M_PI * M_PI)));
  KC_TRY(upload(op->dcl_d, dcl));
  op->kvec.assign(k_host, k_host + 3 * (size_t)nk);
  op->gamma = gam;
  op->smin = smin;
  op->smax = smax;
  op->kflags = kfl;
  op->dcl = dcl;
  op->nk = nk;
  return KC_OK;
}

int kc_get_gamma(const kc_op* op, double* gamma_host) {
  KC_ARG(op != nullptr && gamma_host != nullptr, "NULL argument");
  for (int i = 0; i < op->nk; ++i) gamma_host[i] = op->gamma[i];
  return KC_OK;
}

int kc_op_flags(const kc_op* op, int* flags_host) {
  KC_ARG(op != nullptr && flags_host != nullptr, "NULL argument");
  *flags_host = op->flags;
  return KC_OK;
}

int kc_kpoint_flags(const kc_op* op, int* flags_host) {
  KC_ARG(op != nullptr && flags_host != nullptr, "NULL argument");
  for (int i = 0; i < op->nk; ++i) flags_host[i] = op->kflags[i];
  return KC_OK;
}

int kc_spurious_bound(const kc_op* op, double* bound_host) {
  KC_ARG(op != nullptr && bound_host != nullptr, "NULL argument");
  for (int i = 0; i < op->nk; ++i) bound_host[i] = op->gamma[i] * op->smin[i];
  return KC_OK;
}

int kc_apply(kc_op* op, int ik0, int nvec, int vecs_per_k, const void* x, void* y, int prec, void* stream) {
  KC_ARG(op != nullptr, "op is NULL");
  KC_ARG(op->nk > 0, "no k-points set");
  KC_ARG(nvec >= 0 && vecs_per_k >= 1, "nvec >= 0, vecs_per_k >= 1");
  KC_ARG(prec == KC_PREC_FP64 || prec == KC_PREC_FP32, "prec");
  if (nvec == 0) return KC_OK;
  KC_ARG(x != nullptr && y != nullptr && x != y, "x, y must be distinct device buffers");
  KC_ARG(ik0 >= 0 && ik0 + (nvec - 1) / vecs_per_k < op->nk, "k-point index out of range");
  VecMap vm;
  vm.vpk = vecs_per_k;
  vm.kstride = vecs_per_k;
  return apply_op(op, ik0, nvec, vm, (const c64*)x, (c64*)y, prec, (hipStream_t)stream);
}

int kc_apply_timed(kc_op* op, int ik0, int nvec, int vecs_per_k, const void* x, void* y, int prec, void* stream,
                   double* pass_ms_host, int* npass_host) {
  KC_ARG(op != nullptr && pass_ms_host != nullptr && npass_host != nullptr, "NULL argument");
  KC_ARG(op->nk > 0 && nvec >= 1 && vecs_per_k >= 1, "nvec >= 1, vecs_per_k >= 1, k-points set");
  KC_ARG(prec == KC_PREC_FP64 || prec == KC_PREC_FP32, "prec");
  KC_ARG(x != nullptr && y != nullptr && x != y, "x, y must be distinct device buffers");
  KC_ARG(ik0 >= 0 && ik0 + (nvec - 1) / vecs_per_k < op->nk, "k-point index out of range");
  const int np = (op->scheme == KC_EPS_CROSSDOF) ? 6 : 5;
  hipEvent_t ev[7];
  for (int i = 0; i <= np; ++i) KC_HIP(hipEventCreate(&ev[i]));
  VecMap vm;
  vm.vpk = vecs_per_k;
  vm.kstride = vecs_per_k;
  int st = apply_op(op, ik0, nvec, vm, (const c64*)x, (c64*)y, prec, (hipStream_t)stream, ev);
  if (st == KC_OK) {
    hipError_t e = hipEventSynchronize(ev[np]);
    for (int i = 0; i < np && e == hipSuccess; ++i) {
      float ms = 0.f;
      e = hipEventElapsedTime(&ms, ev[i], ev[i + 1]);
      pass_ms_host[i] = ms;
    }
    if (e != hipSuccess) {
      set_error(std::string("event timing: ") + hipGetErrorString(e));
      st = KC_ERR_HIP;
    }
    *npass_host = np;
  }
  for (int i = 0; i <= np; ++i) (void)hipEventDestroy(ev[i]);
  return st;
}

int kc_precond(kc_op* op, int ik0, int nvec, int vecs_per_k, const void* r, void* z, void* stream) {
  KC_ARG(op != nullptr, "op is NULL");
  KC_ARG(op->nk > 0, "no k-points set");
  KC_ARG(nvec >= 0 && vecs_per_k >= 1, "nvec >= 0, vecs_per_k >= 1");
  if (nvec == 0) return KC_OK;
  KC_ARG(r != nullptr && z != nullptr, "NULL vector");
  KC_ARG(ik0 >= 0 && ik0 + (nvec - 1) / vecs_per_k < op->nk, "k-point index out of range");
  return apply_precond(op, ik0, nvec, vecs_per_k, (const c64*)r, (c64*)z, (hipStream_t)stream);
}

int kc_precond_transverse(kc_op* op, int ik0, int nvec, int vecs_per_k, const void* r, void* z,
                          const float* efield, int prec, void* stream) {
  KC_ARG(op != nullptr, "op is NULL");
  KC_ARG(op->nk > 0, "no k-points set");
  KC_ARG(nvec >= 0 && vecs_per_k >= 1, "nvec >= 0, vecs_per_k >= 1");
  KC_ARG(prec == KC_PREC_FP64 || prec == KC_PREC_FP32, "prec");
  if (nvec == 0) return KC_OK;
  KC_ARG(r != nullptr && z != nullptr, "NULL vector");
  KC_ARG(ik0 >= 0 && ik0 + (nvec - 1) / vecs_per_k < op->nk, "k-point index out of range");
  const size_t n = 3 * (size_t)op->N * op->N * op->N;
  KC_ARG((const char*)z + nvec * n * sizeof(c64) <= (const char*)r ||
             (const char*)r + nvec * n * sizeof(c64) <= (const char*)z,
         "r and z must not overlap");
  KC_TRY(build_efield(op));
  VecMap vm;
  vm.vpk = vecs_per_k;
  vm.kstride = vecs_per_k;
  return apply_tp(op, ik0, nvec, vm, vm, (const c64*)r, (c64*)z, efield ? efield : op->efield.as<float>(),
                  efield ? 1 : 0, prec, (hipStream_t)stream);
}

int kc_tp_grad(kc_op* op, int ik0, int nvec, int vecs_per_k, const void* r, const void* e, const double* w,
               float* g, void* stream) {
  KC_ARG(op != nullptr && op->nk > 0, "op with k-points");
  KC_ARG(nvec >= 1 && vecs_per_k >= 1 && nvec % vecs_per_k == 0, "nvec a positive multiple of vecs_per_k");
  KC_ARG(r != nullptr && e != nullptr && w != nullptr && g != nullptr, "NULL argument");
  KC_ARG(ik0 >= 0 && ik0 + nvec / vecs_per_k <= op->nk, "k-point index out of range");
  return tp_grad(op, ik0, nvec, vecs_per_k, (const c64*)r, (const c64*)e, w, g, (hipStream_t)stream);
}

int kc_fft3d(int N, int nvec, int sign, int prec, const void* in, void* out, void* stream) {
  if (!supported_n(N)) {
    set_error("unsupported N");
    return KC_ERR_UNSUPPORTED;
  }
  KC_ARG(nvec >= 0, "nvec");
  KC_ARG(sign == 1 || sign == -1, "sign must be +1 or -1");
  KC_ARG(prec == KC_PREC_FP64 || prec == KC_PREC_FP32, "prec");
  if (nvec == 0) return KC_OK;
  KC_ARG(in != nullptr && out != nullptr, "NULL buffer");
  int dev = 0;
  KC_HIP(hipGetDevice(&dev));
  DevBuf* tb = nullptr;
  {
    TwCache& c = twcache();
    std::lock_guard<std::mutex> lk(c.mu);
    auto it = c.tabs.find({dev, N});
    if (it == c.tabs.end()) {
      std::vector<c64> d;
      std::vector<c32> f;
      make_twiddles(N, d, f);
      tb = new DevBuf();
      KC_TRY(tb->ensure(N * (sizeof(c64) + sizeof(c32))));
      KC_HIP(hipMemcpy(tb->p, d.data(), N * sizeof(c64), hipMemcpyHostToDevice));
      KC_HIP(hipMemcpy((char*)tb->p + N * sizeof(c64), f.data(), N * sizeof(c32), hipMemcpyHostToDevice));
      c.tabs[{dev, N}] = tb;
    } else {
      tb = it->second;
    }
  }
  const void* tw = (prec == KC_PREC_FP64) ? tb->p : (const void*)((const char*)tb->p + N * sizeof(c64));
  return fft3d(N, nvec, sign, prec, in, out, tw, (hipStream_t)stream);
}

int kc_tile_widths(const kc_op* op, int prec, int* widths_host) {
  KC_ARG(op != nullptr && widths_host != nullptr, "NULL argument");
  KC_ARG(prec == KC_PREC_FP64 || prec == KC_PREC_FP32, "prec");
  const int pi = prec == KC_PREC_FP64 ? 1 : 0;
  for (int i = 0; i < TP_NPASS; ++i) widths_host[i] = op->tuned[pi] ? op->tiles[pi][i] : 0;
  return KC_OK;
}

int kc_last_solve_stats(const kc_op* op, double* stats_host) {
  KC_ARG(op != nullptr && stats_host != nullptr, "NULL argument");
  for (int i = 0; i < 8; ++i) stats_host[i] = op->stats[i];
  return KC_OK;
}

int kc_release_workspaces(kc_op* op) {
  KC_ARG(op != nullptr, "op is NULL");
  KC_HIP(hipDeviceSynchronize());
  solver_release(op);
  op->work_a.release();
  op->work_b.release();
  op->work_c.release();
  op->work_k.release();
  op->efield_k.release();
  op->efield_kt.release();
  op->train_buf.release();
  return KC_OK;
}

void kc_destroy(kc_op* op) {
  if (!op) return;
  // a caller allocator may hand the memory to other work as soon as it is freed
  if (op->alloc.free != nullptr) (void)hipDeviceSynchronize();
  solver_release(op);
  delete op;
}

static int to_space(kc_op* op, int nvec, const void* in, void* out, int sign, void* stream) {
  KC_ARG(op != nullptr, "op is NULL");
  KC_ARG(nvec >= 0, "nvec >= 0");
  if (nvec == 0) return KC_OK;
  KC_ARG(in != nullptr && out != nullptr, "NULL vector");
  const int N = op->N;
  const size_t N3 = (size_t)N * N * N;
  hipStream_t s = (hipStream_t)stream;
  KC_TRY(fft3d(N, 3 * nvec, sign, KC_PREC_FP64, in, out, op->tw64.p, s));
  const size_t total = 3 * (size_t)nvec * N3;
  k_scale<<<(unsigned)std::min<size_t>((total + 255) / 256, 65536), 256, 0, s>>>((c64*)out, total,
                                                                                1.0 / std::sqrt((double)N3));
  KC_LAUNCHED();
  return KC_OK;
}

int kc_to_real_space(kc_op* op, int nvec, const void* x, void* H, void* stream) {
  return to_space(op, nvec, x, H, +1, stream);
}

int kc_to_kspace(kc_op* op, int nvec, const void* H, void* x, void* stream) {
  return to_space(op, nvec, H, x, -1, stream);
}

const char* kc_status_string(int status) {
  switch (status) {
    case KC_OK: return "KC_OK";
    case KC_ERR_INVALID_ARG: return "KC_ERR_INVALID_ARG";
    case KC_ERR_UNSUPPORTED: return "KC_ERR_UNSUPPORTED";
    case KC_ERR_NOT_HPD: return "KC_ERR_NOT_HPD";
    case KC_ERR_HIP: return "KC_ERR_HIP";
    case KC_ERR_ALLOC: return "KC_ERR_ALLOC";
    case KC_ERR_NO_CONVERGENCE: return "KC_ERR_NO_CONVERGENCE";
    case KC_ERR_BREAKDOWN: return "KC_ERR_BREAKDOWN";
    default: return "KC_ERR_UNKNOWN";
  }
}

const char* kc_last_error(void) { return get_error(); }

// ---------------------------------------------------------------- learned preconditioner
struct kc_net : kc::Net {};

int kc_net_create(uint64_t seed, kc_net** out) {
  KC_ARG(out != nullptr, "out is NULL");
  kc_net* n = new kc_net();
  int st = nn_init(n, seed);
  if (st != KC_OK) {
    delete n;
    return st;
  }
  *out = n;
  return KC_OK;
}

size_t kc_net_param_count(void) { return nn_param_count(); }

int kc_net_get_params(const kc_net* net, float* host, size_t n) {
  KC_ARG(net != nullptr && host != nullptr && n == nn_param_count(), "net, host buffer and size");
  KC_HIP(hipMemcpy(host, net->params.p, n * sizeof(float), hipMemcpyDeviceToHost));
  return KC_OK;
}

int kc_net_set_params(kc_net* net, const float* host, size_t n) {
  KC_ARG(net != nullptr && host != nullptr && n == nn_param_count(), "net, host buffer and size");
  KC_HIP(hipMemcpy(net->params.p, host, n * sizeof(float), hipMemcpyHostToDevice));
  return nn_pack(net, nullptr);
}

int kc_net_forward(kc_net* net, int N, int batch, const void* in_bf16, void* out_f32, void* stream) {
  KC_ARG(net != nullptr && in_bf16 != nullptr && out_f32 != nullptr, "NULL argument");
  KC_ARG(N >= 16 && N % 16 == 0 && batch >= 1, "N must be a multiple of 16, batch >= 1");
  return nn_forward(net, N, batch, (const uint16_t*)in_bf16, (float*)out_f32, (hipStream_t)stream);
}

int kc_net_gradients(kc_net* net, int N, int batch, const void* in_bf16, const void* target_f32, double* loss_host,
                     float* grads_host, void* stream) {
  KC_ARG(net != nullptr && in_bf16 != nullptr && target_f32 != nullptr, "NULL argument");
  KC_ARG(N >= 16 && N % 16 == 0 && batch >= 1, "N must be a multiple of 16, batch >= 1");
  hipStream_t s = (hipStream_t)stream;
  KC_TRY(nn_gradients(net, N, batch, (const uint16_t*)in_bf16, (const float*)target_f32, loss_host, s));
  if (grads_host) {
    KC_HIP(hipMemcpyAsync(grads_host, net->grads.p, nn_param_count() * sizeof(float), hipMemcpyDeviceToHost, s));
    KC_HIP(hipStreamSynchronize(s));
  }
  return KC_OK;
}

int kc_net_backward(kc_net* net, int N, int batch, const void* in_bf16, const void* gout_f32, float* grads_host,
                    void* stream) {
  KC_ARG(net != nullptr && in_bf16 != nullptr && gout_f32 != nullptr, "NULL argument");
  KC_ARG(N >= 16 && N % 16 == 0 && batch >= 1, "N must be a multiple of 16, batch >= 1");
  hipStream_t s = (hipStream_t)stream;
  KC_TRY(nn_backward(net, N, batch, (const uint16_t*)in_bf16, (const float*)gout_f32, s));
  if (grads_host) {
    KC_HIP(hipMemcpyAsync(grads_host, net->grads.p, nn_param_count() * sizeof(float), hipMemcpyDeviceToHost, s));
  }
  KC_HIP(hipStreamSynchronize(s));
  return KC_OK;
}

int kc_net_adam_step(kc_net* net, float lr, float beta1, float beta2, float eps, void* stream) {
  KC_ARG(net != nullptr && lr > 0.f, "net and lr > 0");
  return nn_adam(net, lr, beta1, beta2, eps, (hipStream_t)stream);
}

void kc_net_destroy(kc_net* net) { delete net; }

int kc_attach_net(kc_op* op, kc_net* net) {
  KC_ARG(op != nullptr, "op is NULL");
  if (net) KC_ARG(op->N % 16 == 0, "the learned preconditioner needs N % 16 == 0");
  op->net = net;
  if (net && op->epsfeat.p == nullptr) KC_TRY(nn_build_eps_features(op));
  if (net) KC_TRY(build_efield(op));
  return KC_OK;
}

int kc_net_features(kc_op* op, int ik0, int nk, void* feat_bf16, void* stream) {
  KC_ARG(op != nullptr && op->N % 16 == 0, "op with N % 16 == 0");
  KC_ARG(nk >= 1 && feat_bf16 != nullptr, "arguments");
  KC_ARG(ik0 >= 0 && ik0 + nk <= op->nk, "k-point index out of range");
  return nn_features(op, ik0, nk, (uint16_t*)feat_bf16, (hipStream_t)stream);
}

int kc_net_efield(kc_op* op, int ik0, int nk, float* efield, void* stream) {
  KC_ARG(op != nullptr && op->net != nullptr, "op with an attached network");
  KC_ARG(nk >= 1 && efield != nullptr, "arguments");
  KC_ARG(ik0 >= 0 && ik0 + nk <= op->nk, "k-point index out of range");
  return nn_efield(op, ik0, nk, efield, (hipStream_t)stream);
}

int kc_precond_learned(kc_op* op, int ik0, int nvec, int vecs_per_k, const void* r, void* z, int prec,
                       void* stream) {
  KC_ARG(op != nullptr && op->net != nullptr, "op with an attached network");
  KC_ARG(op->nk > 0 && nvec >= 1 && vecs_per_k >= 1 && r != nullptr && z != nullptr, "arguments");
  KC_ARG(prec == KC_PREC_FP64 || prec == KC_PREC_FP32, "prec");
  KC_ARG(ik0 >= 0 && ik0 + (nvec - 1) / vecs_per_k < op->nk, "k-point index out of range");
  const size_t n = 3 * (size_t)op->N * op->N * op->N;
  KC_ARG((const char*)z + nvec * n * sizeof(c64) <= (const char*)r ||
             (const char*)r + nvec * n * sizeof(c64) <= (const char*)z,
         "r and z must not overlap");
  hipStream_t s = (hipStream_t)stream;
  const int nk = (nvec - 1) / vecs_per_k + 1;
  KC_TRY(learned_fields(op, ik0, nk, s));
  VecMap vm;
  vm.vpk = vecs_per_k;
  vm.kstride = vecs_per_k;
  return apply_tp(op, ik0, nvec, vm, vm, (const c64*)r, (c64*)z, op->efield_k.as<float>(), 1, prec, s);
}

size_t kc_block_work_bytes(int nb, size_t n, int nc) {
  if (nb < 1 || n < 1 || nc < 1 || nc > RR_NMAX_WIDE) return 0;
  const size_t upd = (size_t)nb * (RR_NMAX_WIDE / 3) * update_grid_x(n, nb) * 2 * sizeof(double);
  return std::max(gram2_part_bytes(nc, n, nb), upd);
}

// Partial sums of kc_block_gram_noalloc: a fixed array per device, held until the process ends.
// Host code never passes `scratch` itself (on the host it names a stand-in, not device memory):
// the device address comes from hipGetSymbolAddress, once per device.
static __device__ __align__(256) unsigned char scratch[KC_NOALLOC_SCRATCH_BYTES];

static int scratch_address(void** out) {
  static std::mutex mu;
  static std::map<int, void*> addr;  // device -> address of its copy of `scratch`
  int dev = 0;
  KC_HIP(hipGetDevice(&dev));
  std::lock_guard<std::mutex> lk(mu);
  auto it = addr.find(dev);
  if (it == addr.end()) {
    void* p = nullptr;
    KC_HIP(hipGetSymbolAddress(&p, HIP_SYMBOL(scratch)));
    if (p == nullptr) {
      set_error("hipGetSymbolAddress returned NULL for the scratch array");
      return KC_ERR_HIP;
    }
    it = addr.emplace(dev, p).first;
  }
  *out = it->second;
  return KC_OK;
}

static bool disjoint(const void* a, size_t na, const void* b, size_t nb) {
  return (const char*)a + na <= (const char*)b || (const char*)b + nb <= (const char*)a;
}

int kc_block_gram(int nb, size_t n, int nc, const void* S, const void* AS, void* GA, void* GB, void* work,
                  size_t work_bytes, void* stream) {
  KC_ARG(nb >= 0 && n >= 1 && nc >= 1 && nc <= RR_NMAX_WIDE, "nb >= 0, n >= 1, 1 <= nc <= 96");
  if (nb == 0) return KC_OK;
  KC_ARG(S != nullptr && AS != nullptr && GA != nullptr && GB != nullptr && work != nullptr, "NULL buffer");
  KC_ARG(work_bytes >= gram2_part_bytes(nc, n, nb), "work_bytes below kc_block_work_bytes");
  return gram2((const c64*)S, (const c64*)AS, nc, nc, n, nb, (c64*)work, (c64*)GA, (c64*)GB, nullptr,
               (hipStream_t)stream);
}

int kc_block_gram_noalloc(int nb, size_t n, int nc, const void* S, const void* AS, void* GA, void* GB,
                          void* stream) {
  KC_ARG(nb >= 0 && n >= 1 && nc >= 1 && nc <= RR_NMAX_WIDE, "nb >= 0, n >= 1, 1 <= nc <= 96");
  if (nb == 0) return KC_OK;
  KC_ARG(S != nullptr && AS != nullptr && GA != nullptr && GB != nullptr, "NULL buffer");
  const size_t T = (size_t)(nc + 15) / 16;
  KC_ARG((size_t)nb * T * (T + 1) * 256 * sizeof(c64) <= KC_NOALLOC_SCRATCH_BYTES,
         "nb * ceil(nc/16) * (ceil(nc/16) + 1) * 4096 must not exceed KC_NOALLOC_SCRATCH_BYTES");
  void* part = nullptr;
  KC_TRY(scratch_address(&part));
  // every partial sum is written by the product kernel before the reduction reads it, so the
  // array needs no clearing between calls
  return gram2_bounded((const c64*)S, (const c64*)AS, nc, n, nb, (c64*)part, KC_NOALLOC_SCRATCH_BYTES, (c64*)GA,
                       (c64*)GB, (hipStream_t)stream);
}

int kc_block_update(int nb, size_t n, int mb, void* S, void* AS, const void* C, const double* theta, void* R,
                    double* res, double* xnorm2, void* work, size_t work_bytes, void* stream) {
  KC_ARG(nb >= 0 && n >= 1 && mb >= 1 && 3 * mb <= RR_NMAX_WIDE, "nb >= 0, n >= 1, 1 <= mb <= 32");
  if (nb == 0) return KC_OK;
  KC_ARG(S != nullptr && AS != nullptr && C != nullptr && theta != nullptr && R != nullptr && res != nullptr &&
             xnorm2 != nullptr && work != nullptr,
         "NULL buffer");
  const size_t sb = (size_t)nb * 3 * mb * n * sizeof(c64), rb = (size_t)nb * mb * n * sizeof(c64);
  KC_ARG(disjoint(S, sb, AS, sb) && disjoint(R, rb, S, sb) && disjoint(R, rb, AS, sb),
         "S, AS and R must not overlap");
  KC_ARG(work_bytes >= (size_t)nb * mb * update_grid_x(n, nb) * 2 * sizeof(double),
         "work_bytes below kc_block_work_bytes");
  KC_TRY(update_res_prepare());
  return update_res((c64*)S, (c64*)AS, 3 * mb, mb, (const c64*)C, n, nb, theta, (c64*)R, (double*)work, res,
                    xnorm2, nullptr, (hipStream_t)stream);
}

}  // extern "C"
