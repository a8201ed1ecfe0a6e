// LOBPCG with soft locking (Section 4: custom block solver, convergence test of eq (4.3)) for
// the m smallest positive eigenvalues of the compensated operator, run for a batch of
// k-points in lock-step (one set of launches per step for the whole batch).
//
// Per k-point the search space is S = [X W P] (3 mb columns) with images AS = [AX AW AP]:
//   1. R = AX - X Theta, Res_j = |r_j| / |x_j|, W = K_P^{-1} R            (k_resid_precond)
//      (or, after the masks of step 2, W = T_E R with the transverse-projection preconditioner
//      for the columns that get a new direction)
//   2. soft locking: columns with Res_j <= tol (j < m) get no new W; k-points whose
//      m bands all satisfy the test are verified with a fresh FP64 application and retired
//   3. AW = Op W (FP32 while the mixed-precision phase lasts, FP64 after)
//   4. GA = S^H AS, GB = S^H S (one pass over S and AS, MFMA); Rayleigh-Ritz on the pencil
//      scaled to unit diagonal (W is neither normalised nor orthogonalised in the large
//      space: the explicit GB takes care of it): X = S C1, P = S Cp with P orthonormal and
//      orthogonal to X (Cp from the W and P parts of C1); the same coefficients give AX, AP.
// At k = 0 the preconditioner removes the DC frequency from every direction, so the
// constant fields (Prop 2.5 (1)) never enter the search space and the reported eigenvalues
// are the smallest positive ones.
#include <algorithm>
#include <chrono>
#include <cmath>
#include <complex>
#include <cstdio>
#include <vector>

#include "kc_blas.h"
#include "kc_nn.h"

namespace kc {

struct SolverWork {
  DevBuf S, AS;
  DevBuf pw;  // plane-wave start: frequencies (int [nb][mb]) then polarizations (c64 [nb][mb][3])
  DevBuf part_gram, part_res, part_upd;
  DevBuf GA, GB, Cu, Lsave, GApp;
  DevBuf theta, res, xn2;
  DevBuf R, tmask;  // residuals (input of T_E) and the columns that get T_E R
  DevBuf ints;  // xmask, wmask, pmask, pvalid [nb*mb each], kskip, flags, kglobal, wskip [nb each]
  hipStream_t gstream = nullptr;  // private stream of graph-captured solves (default priority)
  void bind_allocator(const Allocator* al) {
    DevBuf* bufs[] = {&S, &AS, &part_gram, &part_res, &part_upd, &GA, &GB, &Cu, &Lsave, &GApp, &theta, &res, &xn2,
                      &R, &tmask, &ints, &pw};
    for (DevBuf* b : bufs) b->al = al;
  }
  ~SolverWork() {
    if (gstream) (void)hipStreamDestroy(gstream);
  }
};

void solver_release(kc_op* op) {
  delete op->solver;
  op->solver = nullptr;
}

namespace {

struct Batch {
  kc_op* op;
  SolverWork* w;
  int ik0, nb, m, mb, nc, N;
  size_t n;
  hipStream_t s;
  int *xmask, *wmask, *pmask, *pvalid, *kskip, *flags, *kglobal, *wskip;
  c64 *S, *AS;
  int pc = KC_PRECOND_DIAG;
  const float* field = nullptr;  // E of T_E: one per k-point (fks = 1) or shared (fks = 0)
  int fks = 0;
};

// The lowest transverse plane waves of k-point ik (the modes of a homogeneous medium): the
// frequencies q with the smallest s(q) = |K(q)|^2 (s = 0, the constant fields at k = 0,
// excluded), with K(q) from the symbol tables (and the lattice terms of eq (2.12)), and for each
// two orthonormal polarizations orthogonal to v = conj(K(q)) (K_A K_A^H + K_B = s I with
// K_B = v v^H, Lemma 2.4 (1)).  Only whole groups of equal s enter (a group cut in two would pick
// an arbitrary part of a degenerate eigenspace), at most ncol columns; q_out [ncol] and
// pol_out [ncol][3], q = -1 for the columns left to the random start.  The frequencies searched
// are those within 4 of 0 on each axis (all of them below N = 10).
void plane_wave_start(const kc_op* op, int ik, int ncol, int* q_out, c64* pol_out) {
  const int N = op->N;
  std::vector<int> ax;
  if (N < 10) {
    for (int q = 0; q < N; ++q) ax.push_back(q);
  } else {
    for (int q = 0; q <= 4; ++q) ax.push_back(q);
    for (int q = N - 4; q < N; ++q) ax.push_back(q);
  }
  struct Cand {
    double s;
    int q;
    std::complex<double> K[3];
  };
  std::vector<Cand> cand;
  const c64* kt = op->ktab_host.data() + (size_t)ik * 3 * N;
  const bool skew = op->skew.l1d != nullptr && !op->lam1_host.empty();
  double smax = 0.0;
  for (int qz : ax)
    for (int qy : ax)
      for (int qx : ax) {
        const int qq[3] = {qx, qy, qz};
        Cand c;
        c.s = 0.0;
        c.q = qx + N * (qy + N * qz);
        for (int i = 0; i < 3; ++i) {
          std::complex<double> Ki(kt[i * N + qq[i]].re, kt[i * N + qq[i]].im);
          if (skew)
            for (int j = 0; j < 3; ++j)
              Ki += op->skew.c[i * 3 + j] * std::complex<double>(op->lam1_host[qq[j]].re, op->lam1_host[qq[j]].im);
          c.K[i] = Ki;
          c.s += std::norm(Ki);
        }
        smax = std::max(smax, c.s);
        cand.push_back(c);
      }
  std::stable_sort(cand.begin(), cand.end(), [](const Cand& a, const Cand& b) { return a.s < b.s; });
  // drop s = 0, then keep whole groups of equal s (two columns per frequency) within ncol
  cand.erase(std::remove_if(cand.begin(), cand.end(), [&](const Cand& c) { return c.s <= 1e-14 * smax; }),
             cand.end());
  size_t keep = 0;
  for (size_t g = 0; g < cand.size();) {
    size_t e = g + 1;
    while (e < cand.size() && cand[e].s - cand[g].s <= 1e-9 * cand[g].s) ++e;
    if (2 * e > (size_t)ncol) break;
    keep = e;
    g = e;
  }
  cand.resize(keep);
  int col = 0;
  for (const Cand& c : cand) {
    const double kn = std::sqrt(c.s);
    std::complex<double> v[3];
    for (int i = 0; i < 3; ++i) v[i] = std::conj(c.K[i]) / kn;
    // the two axes where v is smallest: e_a, e_b minus their projections give the basis
    int o[3] = {0, 1, 2};
    std::sort(o, o + 3, [&](int x, int y) { return std::abs(v[x]) < std::abs(v[y]); });
    std::complex<double> u[2][3];
    for (int t = 0; t < 2; ++t) {
      const int a = o[t];
      for (int i = 0; i < 3; ++i) u[t][i] = (i == a ? 1.0 : 0.0) - v[i] * std::conj(v[a]);
      if (t == 1) {
        std::complex<double> d(0.0, 0.0);
        for (int i = 0; i < 3; ++i) d += std::conj(u[0][i]) * u[1][i];
        for (int i = 0; i < 3; ++i) u[1][i] -= d * u[0][i];
      }
      double nn = 0.0;
      for (int i = 0; i < 3; ++i) nn += std::norm(u[t][i]);
      nn = std::sqrt(nn);
      for (int i = 0; i < 3; ++i) u[t][i] /= nn;
    }
    for (int t = 0; t < 2 && col < ncol; ++t, ++col) {
      q_out[col] = c.q;
      for (int i = 0; i < 3; ++i) pol_out[(size_t)col * 3 + i] = mk(u[t][i].real(), u[t][i].imag());
    }
  }
  for (; col < ncol; ++col) {
    q_out[col] = -1;
    for (int i = 0; i < 3; ++i) pol_out[(size_t)col * 3 + i] = mk(0.0, 0.0);
  }
}

int upload_ints(int* dst, const std::vector<int>& v, hipStream_t s) {
  KC_HIP(hipMemcpyAsync(dst, v.data(), v.size() * sizeof(int), hipMemcpyHostToDevice, s));
  return KC_OK;
}

// AX (or AP...) for columns [col0, col0+mb) of every k-point in the batch, masked by `active`
int apply_cols(Batch& B, int col0, const int* active, int prec) {
  VecMap vm;
  vm.vpk = B.mb;
  vm.kstride = B.nc;
  vm.active = active;
  return apply_op(B.op, B.ik0, B.nb * B.mb, vm, B.S + (size_t)col0 * B.n, B.AS + (size_t)col0 * B.n, prec, B.s);
}

// Gram matrices (all blocks, or with `implicit` only the W columns, the X/P blocks coming from
// the previous step), small Rayleigh-Ritz, update; with `fused` the update pass also forms the
// next residuals R (for T_E) and their norms
int rayleigh_ritz(Batch& B, bool implicit = false, bool fused = false) {
  if (implicit) {
    KC_TRY(gramw(B.S, B.AS, B.nc, B.mb, B.n, B.nb, B.w->part_gram, B.w->GA.as<c64>(), B.w->GB.as<c64>(),
                 B.w->theta.as<double>(), B.w->GApp.as<c64>(), B.kskip, B.s));
  } else {
    KC_TRY(gram2(B.S, B.AS, B.nc, B.nc, B.n, B.nb, B.w->part_gram, B.w->GA.as<c64>(), B.w->GB.as<c64>(),
                 B.kskip, B.s));
  }
  KC_TRY(small_rr(B.w->GA.as<c64>(), B.w->GB.as<c64>(), B.mb, B.nb, B.xmask, B.wmask, B.pmask,
                  B.w->theta.as<double>(), B.w->Cu.as<c64>(), B.pvalid, B.w->Lsave.as<c64>(), B.flags, B.kskip,
                  B.w->GApp.as<c64>(), B.s, B.w->res.as<double>()));
  // [X | P] <- S Cu, [AX | AP] <- AS Cu
  if (fused)
    return update_res(B.S, B.AS, B.nc, B.mb, B.w->Cu.as<c64>(), B.n, B.nb, B.w->theta.as<double>(),
                      B.w->R.as<c64>(), B.w->part_upd.as<double>(), B.w->res.as<double>(), B.w->xn2.as<double>(),
                      B.kskip, B.s);
  KC_TRY(update(B.S, B.nc, 0, B.nc, B.S, B.nc, 2 * B.mb, B.mb, 0, 2 * B.mb, B.w->Cu.as<c64>(), B.n, B.nb,
                B.kskip, B.s));
  KC_TRY(update(B.AS, B.nc, 0, B.nc, B.AS, B.nc, 2 * B.mb, B.mb, 0, 2 * B.mb, B.w->Cu.as<c64>(), B.n, B.nb,
                B.kskip, B.s));
  return KC_OK;
}

// The new directions W of the k-points near Gamma whose DC longitudinal direction is deflated
// (kc_set_kpoints) lose that component, so the search space never holds it.
int deflate_w(Batch& B) {
  return deflate_dc_long(B.S, B.nc, B.mb, B.mb, B.nb, B.op->ktab64.as<c64>() + (size_t)B.ik0 * 3 * B.N, B.N,
                         B.op->dcl_d.as<int>() + B.ik0, B.s);
}

// Res and W = K_P^{-1} R; with copy_r also a contiguous copy of R for T_E, and W = K_P^{-1} R
// only for the k-points that do not use T_E (wskip)
int residuals(Batch& B, bool copy_r) {
  c64* R = copy_r ? B.w->R.as<c64>() : nullptr;
  KC_TRY(resid_precond(B.S, B.AS, B.S, B.w->theta.as<double>(), B.op->ktab64.as<c64>() + (size_t)B.ik0 * 3 * B.N,
                       B.op->gamma_d.as<double>() + B.ik0, B.N, B.nc, 0, B.mb, B.mb, B.nb, B.w->part_res,
                       B.w->res.as<double>(), B.w->xn2.as<double>(), B.kskip, B.s, R, nullptr,
                       copy_r ? B.wskip : nullptr, B.op->sfloor_d.as<double>() + B.ik0, &B.op->skew));
  return deflate_w(B);
}

// W = T_E R (FP32 transforms) for the columns whose tmask is set; the others keep K_P^{-1} R
int precond_tp(Batch& B) {
  VecMap vx, vy;
  vx.vpk = vy.vpk = B.mb;
  vx.kstride = B.mb;
  vy.kstride = B.nc;
  vx.active = vy.active = B.w->tmask.as<int>();
  KC_TRY(apply_tp(B.op, B.ik0, B.nb * B.mb, vx, vy, B.w->R.as<c64>(), B.S + (size_t)B.mb * B.n, B.field, B.fks,
                  KC_PREC_FP32, B.s, B.op->sfloor_d.as<double>()));
  return deflate_w(B);
}

// Rounding floor of an FP32 operator application on the k-points ik0 .. ik0+nb-1, as an absolute
// residual of a unit vector: the FP32 transforms round at 2^-24 of the largest values they carry,
// and the curl-(eps^-1)-curl part of Op reaches s_max |eps^-1| (largest s(p) of the k-points
// times the largest absolute row sum of eps^-1 over the materials the grid uses, which bounds
// its norm); the penalty term is formed in FP64 and adds nothing.
double fp32_floor(const kc_op* op, int ik0, int nb) {
  double smx = 0.0;
  for (int b = 0; b < nb; ++b) smx = std::max(smx, op->smax[ik0 + b]);
  return std::ldexp(smx * op->epsinv_norm, -24);
}

int solve_batch(kc_op* op, int ik0, int nb, const kc_solve_opts& o, double* eig, double* res_out, int* iters,
                c64* Xout, const c64* xinit, hipStream_t s, bool* all_conv) {
  if (!op->solver) op->solver = new SolverWork();
  SolverWork* w = op->solver;
  w->bind_allocator(&op->alloc);
  Batch B;
  B.op = op;
  B.w = w;
  B.ik0 = ik0;
  B.nb = nb;
  B.m = o.m;
  B.mb = o.m + o.guard;
  B.nc = 3 * B.mb;
  B.N = op->N;
  B.n = 3 * (size_t)op->N * op->N * op->N;
  B.s = s;
  const int mb = B.mb, nc = B.nc, m = B.m;
  const size_t n = B.n;
  const size_t colbytes = n * sizeof(c64);
  KC_TRY(w->S.ensure((size_t)nb * nc * colbytes));
  KC_TRY(w->AS.ensure((size_t)nb * nc * colbytes));
  KC_TRY(w->GA.ensure((size_t)nb * nc * nc * sizeof(c64)));
  KC_TRY(w->GB.ensure((size_t)nb * nc * nc * sizeof(c64)));
  KC_TRY(w->Cu.ensure((size_t)nb * nc * 2 * mb * sizeof(c64)));
  KC_TRY(w->Lsave.ensure((size_t)nb * small_rr_ws_bytes(mb)));
  KC_TRY(w->GApp.ensure((size_t)nb * mb * mb * sizeof(c64)));
  KC_TRY(w->theta.ensure((size_t)nb * mb * sizeof(double)));
  KC_TRY(w->res.ensure((size_t)nb * mb * sizeof(double)));
  KC_TRY(w->xn2.ensure((size_t)nb * mb * sizeof(double)));
  B.pc = o.precond;
  const bool tp = B.pc != KC_PRECOND_DIAG;
  if (B.pc == KC_PRECOND_LEARNED) {
    if (!op->net) {
      set_error("learned preconditioner requested but no network is attached");
      return KC_ERR_INVALID_ARG;
    }
    // one network pass per k-point of the batch gives its field
    KC_TRY(learned_fields(op, ik0, nb, s));
    B.field = op->efield_k.as<float>();
    B.fks = 1;
  } else if (B.pc == KC_PRECOND_TRANSVERSE) {
    KC_TRY(build_efield(op));
    B.field = op->efield.as<float>();
    B.fks = 0;
  }
  if (tp) {
    KC_TRY(w->R.ensure((size_t)nb * mb * colbytes));
    KC_TRY(w->tmask.ensure((size_t)nb * mb * sizeof(int)));
  }
  // with T_E on every k-point the update pass forms the next residuals itself (the learned
  // field falls back to K_P^{-1} per k-point, which needs the separate residual pass)
  const bool fused = B.pc == KC_PRECOND_TRANSVERSE;
  if (fused) {
    KC_TRY(w->part_upd.ensure((size_t)nb * mb * update_grid_x(n, nb) * 2 * sizeof(double)));
    KC_TRY(update_res_prepare());
  }
  KC_TRY(w->ints.ensure((size_t)(4 * nb * mb + 4 * nb) * sizeof(int)));
  // operator work buffers at their largest (FP64) size up front: captured iterations keep
  // their pointers, so no buffer may move after a capture
  KC_TRY(op->work_a.ensure((size_t)nb * mb * n * sizeof(c64)));
  if (op->scheme == KC_EPS_CROSSDOF) KC_TRY(op->work_b.ensure((size_t)nb * mb * n * sizeof(c64)));
  KC_TRY(op->work_k.ensure((size_t)nb * mb * (n / 3) * sizeof(c64)));
  B.S = w->S.as<c64>();
  B.AS = w->AS.as<c64>();
  int* ib = w->ints.as<int>();
  B.xmask = ib;
  B.wmask = ib + nb * mb;
  B.pmask = ib + 2 * nb * mb;
  B.pvalid = ib + 3 * nb * mb;
  B.kskip = ib + 4 * nb * mb;
  B.flags = B.kskip + nb;
  B.kglobal = B.flags + nb;
  B.wskip = B.kglobal + nb;

  std::vector<int> hx(nb * mb, 0), hw(nb * mb, 1), hp(nb * mb, 0), hpv(nb * mb, 0), hskip(nb, 0), hflags(nb, 0),
      hkg(nb);
  for (int b = 0; b < nb; ++b) hkg[b] = ik0 + b;
  std::vector<double> hres(nb * mb, 0.0), htheta(nb * mb, -1.0);
  std::vector<char> done(nb, 0);
  std::vector<int> its(nb, 0), brk_count(nb, 0);
  std::vector<char> drop_p(nb, 0);
  std::vector<double> sbest(nb, 1e300);
  std::vector<int> sstall(nb, 0), sgrow(nb, 0);
  std::vector<char> stalled(nb, 0);

  KC_HIP(hipMemsetAsync(B.S, 0, (size_t)nb * nc * colbytes, s));
  KC_HIP(hipMemsetAsync(B.AS, 0, (size_t)nb * nc * colbytes, s));
  KC_TRY(upload_ints(B.kglobal, hkg, s));
  KC_TRY(upload_ints(B.kskip, hskip, s));
  KC_TRY(upload_ints(B.flags, hflags, s));
  KC_TRY(upload_ints(B.pvalid, hpv, s));
  // initial block: W = K_P^{-1} (random), using the residual pass with AX = 0, theta = -1
  KC_TRY(random_block(B.S, n, nc, 0, mb, nb, o.seed, B.kglobal, s));
  KC_HIP(hipMemcpyAsync(w->theta.p, htheta.data(), htheta.size() * sizeof(double), hipMemcpyHostToDevice, s));
  KC_TRY(residuals(B, false));
  if (!xinit && o.start == KC_START_PLANE_WAVES) {
    // the lowest transverse plane waves of each k-point (whole degenerate groups, up to mb
    // columns) replace the first new directions of the first step; the others stay random
    std::vector<int> hq((size_t)nb * mb);
    std::vector<c64> hpol((size_t)nb * mb * 3);
    for (int b = 0; b < nb; ++b)
      plane_wave_start(op, ik0 + b, mb, hq.data() + (size_t)b * mb, hpol.data() + (size_t)b * mb * 3);
    const size_t qbytes = (hq.size() * sizeof(int) + 15) / 16 * 16;  // the polarizations start aligned
    KC_TRY(w->pw.ensure(qbytes + hpol.size() * sizeof(c64)));
    c64* dpol = reinterpret_cast<c64*>(w->pw.as<char>() + qbytes);
    KC_HIP(hipMemcpyAsync(w->pw.p, hq.data(), hq.size() * sizeof(int), hipMemcpyHostToDevice, s));
    KC_HIP(hipMemcpyAsync(dpol, hpol.data(), hpol.size() * sizeof(c64), hipMemcpyHostToDevice, s));
    KC_HIP(hipStreamSynchronize(s));
    KC_TRY(plane_wave_block(B.S, n, nc, mb, mb, nb, w->pw.as<int>(), dpol, s));
    KC_TRY(deflate_w(B));
  }
  if (xinit) {
    // given start vectors take the first m new directions (the guard columns keep the
    // preconditioned random ones); at k = 0 their DC entries go, as K_P^{-1} would remove them
    const size_t N3 = (size_t)B.N * B.N * B.N;
    for (int b = 0; b < nb; ++b) {
      c64* w0 = B.S + ((size_t)b * nc + mb) * n;
      KC_HIP(hipMemcpyAsync(w0, xinit + (size_t)b * m * n, (size_t)m * colbytes, hipMemcpyDeviceToDevice, s));
      const double* kv = &op->kvec[3 * (size_t)(ik0 + b)];
      if (kv[0] == 0.0 && kv[1] == 0.0 && kv[2] == 0.0)
        for (int j = 0; j < m; ++j)
          for (int c = 0; c < 3; ++c) KC_HIP(hipMemsetAsync(w0 + (size_t)j * n + c * N3, 0, sizeof(c64), s));
    }
    KC_TRY(deflate_w(B));
  }
  // T_E per k-point; with the learned field a k-point falls back to K_P^{-1} when the geometric
  // mean of its band residuals (each floored at tol) stops decreasing or grows
  std::vector<int> lon(nb, tp ? 1 : 0), ht(nb * mb, 0);
  std::vector<double> lbest(nb, 1e300);
  std::vector<int> lstall(nb, 0);
  double napp = 0;
  KC_TRY(upload_ints(B.wskip, lon, s));
  KC_TRY(upload_ints(B.xmask, hx, s));
  KC_TRY(upload_ints(B.wmask, hw, s));
  KC_TRY(upload_ints(B.pmask, hp, s));
  int prec = o.prec;
  bool mixed = (o.prec == KC_PREC_FP32);
  double nmv64 = 0, nmv32 = 0;
  KC_TRY(apply_cols(B, mb, B.wmask, prec));
  (prec == KC_PREC_FP64 ? nmv64 : nmv32) += nb * mb;
  KC_TRY(rayleigh_ritz(B));
  std::fill(hx.begin(), hx.end(), 1);
  KC_TRY(upload_ints(B.xmask, hx, s));

  // One iteration's device work after the masks are uploaded: W = T_E R on the active
  // columns, AW = Op W, Rayleigh-Ritz and update, then the next residuals.  With o.graph it is
  // captured once per precision into a hipGraph and replayed; every launch has a fixed grid
  // (masked columns exit early), reads its masks from device memory and writes to buffers
  // sized before the first capture.
  // With `implicit` the Gram step forms only the W columns (the X/P blocks are known from the
  // previous Rayleigh-Ritz step); that is valid while X, P, AX and AP are the last step's output,
  // so after a fresh application of Op to X or P (precision switch, verification) or a
  // breakdown the next step forms all blocks, and near convergence (Res within 1e4 tol) every
  // step does, where rounding in the assumed blocks would show.
  auto body = [&](int pr, bool implicit) -> int {
    if (tp) KC_TRY(precond_tp(B));
    KC_TRY(apply_cols(B, mb, B.wmask, pr));
    KC_TRY(rayleigh_ritz(B, implicit, fused));
    return fused ? KC_OK : residuals(B, tp);
  };
  hipGraphExec_t gexec[4] = {nullptr, nullptr, nullptr, nullptr};
  struct GraphGuard {
    hipGraphExec_t* g;
    ~GraphGuard() {
      for (int i = 0; i < 4; ++i)
        if (g[i]) (void)hipGraphExecDestroy(g[i]);
    }
  } gguard{gexec};
  auto run_body = [&](int pr, bool implicit) -> int {
    if (!o.graph) return body(pr, implicit);
    const int slot = ((pr == KC_PREC_FP64) ? 1 : 0) + (implicit ? 2 : 0);
    if (!gexec[slot]) {
      KC_HIP(hipStreamBeginCapture(s, hipStreamCaptureModeThreadLocal));
      const int st = body(pr, implicit);
      hipGraph_t g = nullptr;
      const hipError_t e = hipStreamEndCapture(s, &g);
      if (st != KC_OK) {
        if (g) (void)hipGraphDestroy(g);
        return st;
      }
      KC_HIP(e);
      const hipError_t ei = hipGraphInstantiate(&gexec[slot], g, nullptr, nullptr, 0);
      (void)hipGraphDestroy(g);
      KC_HIP(ei);
    }
    KC_HIP(hipGraphLaunch(gexec[slot], s));
    return KC_OK;
  };

  int it = 0;
  double best_max = 1e300;
  // within ten times the FP32 rounding floor, a rise of the largest residual ends the FP32 phase
  const double rise_level = 10.0 * fp32_floor(op, ik0, nb);
  double min_max = 1e300;
  int stall = 0;
  bool verify_pending = false;
  bool need_resid = true;
  bool full_gram = true;  // the next Gram step forms all blocks
  double ngram_w = 0;
  while (true) {
    if (need_resid) KC_TRY(residuals(B, tp));
    need_resid = true;
    KC_HIP(hipMemcpyAsync(hres.data(), w->res.p, hres.size() * sizeof(double), hipMemcpyDeviceToHost, s));
    KC_HIP(hipMemcpyAsync(hpv.data(), B.pvalid, hpv.size() * sizeof(int), hipMemcpyDeviceToHost, s));
    KC_HIP(hipMemcpyAsync(hflags.data(), B.flags, hflags.size() * sizeof(int), hipMemcpyDeviceToHost, s));
    KC_HIP(hipStreamSynchronize(s));
    bool reset_flags = false;
    for (int b = 0; b < nb; ++b) {
      if (done[b]) continue;
      for (int j = 0; j < mb; ++j)
        if (!std::isfinite(hres[b * mb + j])) hflags[b] |= 1;
      if (hflags[b] & 2) {  // a rejected Rayleigh-Ritz step (negative Ritz value): restart from X
        reset_flags = true;
        drop_p[b] = 1;
        full_gram = true;
      }
      if (hflags[b] & 1) {
        reset_flags = true;
        drop_p[b] = 1;
        full_gram = true;
        if (++brk_count[b] > 5) {
          set_error("LOBPCG breakdown (loss of positive definiteness or non-finite values) at k-point " +
                    std::to_string(ik0 + b));
          return KC_ERR_BREAKDOWN;
        }
      }
    }
    if (reset_flags) {
      std::fill(hflags.begin(), hflags.end(), 0);
      KC_TRY(upload_ints(B.flags, hflags, s));
    }
    if (o.verbose) {
      double mx = 0;
      for (int b = 0; b < nb; ++b)
        if (!done[b])
          for (int j = 0; j < m; ++j) mx = std::max(mx, hres[b * mb + j]);
      fprintf(stderr, "[kc_solve] k %d..%d it %d prec %s max res %.3e\n", ik0, ik0 + nb - 1, it,
              prec == KC_PREC_FP64 ? "fp64" : "fp32", mx);
      if (o.verbose > 1) {
        std::vector<double> th(nb * mb);
        KC_HIP(hipMemcpy(th.data(), w->theta.p, th.size() * sizeof(double), hipMemcpyDeviceToHost));
        fprintf(stderr, "   theta:");
        for (int j = 0; j < mb; ++j) fprintf(stderr, " %.10f", th[j]);
        fprintf(stderr, "\n   res:  ");
        for (int j = 0; j < mb; ++j) fprintf(stderr, " %.2e", hres[j]);
        fprintf(stderr, "\n   pval: ");
        for (int j = 0; j < mb; ++j) fprintf(stderr, " %d", hpv[j]);
        fprintf(stderr, " flags %d\n", hflags[0]);
      }
    }
    // verification outcome / convergence test
    std::vector<int> cand(nb, 0);
    int ncand = 0, nlive = 0;
    double mxres = 0.0;
    for (int b = 0; b < nb; ++b) {
      if (done[b]) continue;
      ++nlive;
      bool ok = true;
      for (int j = 0; j < m; ++j) {
        ok = ok && hres[b * mb + j] <= o.tol;
        mxres = std::max(mxres, hres[b * mb + j]);
      }
      if (ok) {
        cand[b] = 1;
        ++ncand;
      }
    }
    bool lchanged = false;
    // the fallback watches the FP64 iterations only: in the FP32 phase the residuals level off at
    // the FP32 floor whatever the preconditioner
    if (B.pc == KC_PRECOND_LEARNED && prec == KC_PREC_FP64) {
      for (int b = 0; b < nb; ++b) {
        if (done[b] || !lon[b]) continue;
        double lg = 0.0;
        for (int j = 0; j < m; ++j) lg += std::log(std::max(hres[b * mb + j], o.tol));
        const double gm = std::exp(lg / m);
        if (gm < 0.95 * lbest[b]) {
          lbest[b] = gm;
          lstall[b] = 0;
        } else if (++lstall[b] >= 8 || gm > 100.0 * lbest[b]) {
          lon[b] = 0;  // fall back to the diagonal-block preconditioner
          lchanged = true;
          if (o.verbose) fprintf(stderr, "[kc_solve] k %d: learned preconditioner off\n", ik0 + b);
        }
      }
      if (lchanged) {  // this iteration's W of those k-points must be K_P^{-1} R
        KC_TRY(upload_ints(B.wskip, lon, s));
        KC_TRY(residuals(B, tp));
      }
    }
    if (verify_pending) {
      // residuals above come from a fresh FP64 application of Op to X
      for (int b = 0; b < nb; ++b)
        if (!done[b] && cand[b]) {
          done[b] = 1;
          its[b] = it;
        }
      verify_pending = false;
      bool any = false;
      for (int b = 0; b < nb; ++b) any = any || !done[b];
      if (!any) break;
      for (int b = 0; b < nb; ++b) hskip[b] = done[b];
      KC_TRY(upload_ints(B.kskip, hskip, s));
      continue;  // recompute residuals/W for the live k-points with the same X
    }
    if (ncand > 0 && prec == KC_PREC_FP64) {
      // fresh FP64 AX for the candidates, then re-test
      std::vector<int> act(nb * mb, 0);
      for (int b = 0; b < nb; ++b)
        if (cand[b])
          for (int j = 0; j < mb; ++j) act[b * mb + j] = 1;
      KC_TRY(upload_ints(B.wmask, act, s));
      KC_TRY(apply_cols(B, 0, B.wmask, KC_PREC_FP64));
      nmv64 += ncand * mb;
      verify_pending = true;
      full_gram = true;
      continue;
    }
    if (it >= o.maxit) break;
    // mixed precision: leave the FP32 phase once the residuals reach switch_tol or stall, or at
    // their first rise near the FP32 rounding floor (there the rounding in AW has begun to steer
    // the Rayleigh-Ritz steps, and waiting for the stall count lets the residuals grow tenfold)
    if (mixed && prec == KC_PREC_FP32) {
      const bool rise = min_max <= rise_level && mxres > min_max;
      min_max = std::min(min_max, mxres);
      if (mxres < best_max * 0.7) {
        best_max = mxres;
        stall = 0;
      } else {
        ++stall;
      }
      if (mxres <= o.switch_tol || stall >= 4 || ncand > 0 || rise) {
        prec = KC_PREC_FP64;
        full_gram = true;
        std::fill(lbest.begin(), lbest.end(), 1e300);
        std::fill(lstall.begin(), lstall.end(), 0);
        std::vector<int> act(nb * mb, 0);
        for (int b = 0; b < nb; ++b)
          if (!done[b])
            for (int j = 0; j < mb; ++j) act[b * mb + j] = 1;
        KC_TRY(upload_ints(B.wmask, act, s));
        KC_TRY(apply_cols(B, 0, B.wmask, KC_PREC_FP64));  // AX
        nmv64 += nlive * mb;
        std::vector<int> pa(nb * mb, 0);
        for (int i = 0; i < nb * mb; ++i) pa[i] = act[i] && hpv[i];
        KC_TRY(upload_ints(B.wmask, pa, s));
        KC_TRY(apply_cols(B, 2 * mb, B.wmask, KC_PREC_FP64));  // AP
        for (int v : pa) nmv64 += v;
        continue;
      }
    }
    // stagnation (FP64 phase): a k-point whose largest band residual has not halved in 200
    // iterations, or that rose above 10 times its best in two successive iterations once within
    // 1e3 tol (past the rounding floor of the operator's FP64 application the running images
    // AX = AS C drift away from Op X and the residuals grow), stops there and is reported as not
    // converged, before the iteration fills the block with rounding noise
    if (prec == KC_PREC_FP64) {
      bool any_live = false;
      for (int b = 0; b < nb; ++b) {
        if (done[b]) continue;
        double mx = 0.0;
        for (int j = 0; j < m; ++j) mx = std::max(mx, hres[b * mb + j]);
        sgrow[b] = (sbest[b] < 1e3 * o.tol && mx > 10.0 * sbest[b]) ? sgrow[b] + 1 : 0;
        if (mx < 0.5 * sbest[b]) {
          sbest[b] = mx;
          sstall[b] = 0;
        } else if (++sstall[b] >= 200 || sgrow[b] >= 2) {
          done[b] = 1;
          stalled[b] = 1;
          its[b] = it;
          if (o.verbose) fprintf(stderr, "[kc_solve] k %d: stagnated at %.3e\n", ik0 + b, sbest[b]);
        }
        any_live = any_live || !done[b];
      }
      if (!any_live) break;
    }
    // masks for this iteration; after a breakdown the k-point restarts without P
    int nact = 0;
    for (int b = 0; b < nb; ++b)
      for (int j = 0; j < mb; ++j) {
        const int i = b * mb + j;
        hw[i] = !done[b] && (j >= m || hres[i] > o.tol);
        // P is kept for locked bands too: its columns are orthonormalised together (each is a
        // mixture of the bands' directions), so dropping one would cut the others
        hp[i] = !done[b] && hpv[i] && !drop_p[b];
        nact += hw[i];
      }
    for (int b = 0; b < nb; ++b) {
      hskip[b] = done[b];
      drop_p[b] = 0;
    }
    KC_TRY(upload_ints(B.wmask, hw, s));
    KC_TRY(upload_ints(B.pmask, hp, s));
    KC_TRY(upload_ints(B.kskip, hskip, s));
    if (tp) {
      int nt = 0;
      for (int b = 0; b < nb; ++b)
        for (int j = 0; j < mb; ++j) {
          const int i = b * mb + j;
          ht[i] = hw[i] && lon[b];
          nt += ht[i];
        }
      KC_TRY(upload_ints(B.w->tmask.as<int>(), ht, s));
      napp += nt;
    }
    // residual history: the largest Res_j (j < m) of every live k-point before this iteration
    for (int b = 0; b < nb; ++b) {
      if (done[b]) continue;
      double mx = 0.0;
      for (int j = 0; j < m; ++j) mx = std::max(mx, hres[b * mb + j]);
      const size_t h = (size_t)(ik0 + b - op->hist_ik0);
      if (h < op->hist.size()) {
        op->hist[h].push_back(mx);
        op->histp[h].push_back((int8_t)prec);
      }
    }
    const bool implicit = !full_gram && mxres > 1e4 * o.tol;
    KC_TRY(run_body(prec, implicit));
    ngram_w += implicit;
    full_gram = false;
    need_resid = false;
    (prec == KC_PREC_FP64 ? nmv64 : nmv32) += nact;
    ++it;
  }
  // results
  std::vector<double> th(nb * mb);
  KC_HIP(hipMemcpyAsync(th.data(), w->theta.p, th.size() * sizeof(double), hipMemcpyDeviceToHost, s));
  KC_HIP(hipStreamSynchronize(s));
  bool allc = true;
  for (int b = 0; b < nb; ++b) {
    for (int j = 0; j < m; ++j) {
      eig[(size_t)b * m + j] = th[b * mb + j];
      res_out[(size_t)b * m + j] = hres[b * mb + j];
    }
    if (iters) iters[b] = done[b] ? its[b] : it;
    allc = allc && done[b] && !stalled[b];
    if (Xout) {
      for (int j = 0; j < m; ++j)
        KC_HIP(hipMemcpyAsync(Xout + ((size_t)b * m + j) * n, B.S + ((size_t)b * nc + j) * n, colbytes,
                              hipMemcpyDeviceToDevice, s));
    }
  }
  KC_HIP(hipStreamSynchronize(s));
  op->stats[0] += nmv64;
  op->stats[1] += nmv32;
  op->stats[3] += (double)it * nb;
  for (int b = 0; b < nb; ++b) op->stats[4] += lon[b];  // k-points that kept T_E to the end
  op->stats[5] += napp;
  op->stats[6] += ngram_w;  // iterations whose Gram step formed only the W columns
  *all_conv = allc;
  return KC_OK;
}

}  // namespace
}  // namespace kc

extern "C" {

void kc_solve_opts_default(kc_solve_opts* o) {
  if (!o) return;
  o->m = 10;
  o->guard = 0;
  o->tol = 1e-8;
  o->maxit = 500;
  o->prec = KC_PREC_FP64;
  o->switch_tol = 1e-3;
  o->batch_k = 1;
  o->seed = 1234;
  o->verbose = 0;
  o->precond = KC_PRECOND_DIAG;
  o->graph = 1;
  o->x_init = nullptr;
  o->start = KC_START_RANDOM;
}

int kc_solve(kc_op* op, int ik0, int nk, const kc_solve_opts* opts, double* eig_host, double* res_host,
             int* iters_host, void* X_out, void* stream) {
  KC_ARG(op != nullptr && opts != nullptr, "NULL op or opts");
  KC_ARG(eig_host != nullptr && res_host != nullptr, "NULL eig or res output");
  KC_ARG(op->nk > 0 && nk >= 1 && ik0 >= 0 && ik0 + nk <= op->nk, "k-point range");
  const kc_solve_opts& o = *opts;
  KC_ARG(o.m >= 1 && o.guard >= 0 && o.m + o.guard <= 32, "m + guard must be in [1, 32]");
  KC_ARG(o.start == KC_START_RANDOM || o.start == KC_START_PLANE_WAVES, "start: KC_START_RANDOM or _PLANE_WAVES");
  KC_ARG((size_t)3 * (o.m + o.guard) <= 3 * (size_t)op->N * op->N * op->N, "block larger than the space");
  KC_ARG(o.tol > 0.0 && o.maxit >= 1 && o.batch_k >= 1, "tol > 0, maxit >= 1, batch_k >= 1");
  KC_ARG(o.prec == KC_PREC_FP64 || o.prec == KC_PREC_FP32, "prec");
  KC_ARG(o.precond == KC_PRECOND_DIAG || o.precond == KC_PRECOND_LEARNED || o.precond == KC_PRECOND_TRANSVERSE,
         "precond");
  hipStream_t s = (hipStream_t)stream;
  if (o.graph) {
    // captured iterations run on a private stream (a capture cannot use the legacy default
    // stream); the solve is synchronous, so ordering with the caller's stream is a sync
    if (!op->solver) op->solver = new kc::SolverWork();
    if (!op->solver->gstream) KC_HIP(hipStreamCreateWithFlags(&op->solver->gstream, hipStreamNonBlocking));
    KC_HIP(hipStreamSynchronize(s));
    s = op->solver->gstream;
  }
  auto t0 = std::chrono::steady_clock::now();
  for (int i = 0; i < 8; ++i) op->stats[i] = 0.0;
  op->hist.assign(nk, {});
  op->histp.assign(nk, {});
  op->hist_ik0 = ik0;
  bool allc = true;
  for (int k0 = 0; k0 < nk; k0 += o.batch_k) {
    const int nb = std::min(o.batch_k, nk - k0);
    bool c = true;
    const size_t vstride = (size_t)k0 * o.m * 3 * op->N * op->N * op->N;
    KC_TRY(kc::solve_batch(op, ik0 + k0, nb, o, eig_host + (size_t)k0 * o.m, res_host + (size_t)k0 * o.m,
                           iters_host ? iters_host + k0 : nullptr, X_out ? (kc::c64*)X_out + vstride : nullptr,
                           o.x_init ? (const kc::c64*)o.x_init + vstride : nullptr, s, &c));
    allc = allc && c;
  }
  KC_HIP(hipStreamSynchronize(s));
  op->stats[2] = std::chrono::duration<double>(std::chrono::steady_clock::now() - t0).count();
  // Prop 2.3: the penalty term's eigenvalues are gamma s(p) >= gamma s_min; the m computed
  // eigenvalues are free of them when the largest lies below that bound
  for (int b = 0; b < nk; ++b) {
    int& f = op->kflags[ik0 + b];
    f &= ~KC_KFLAG_SPURIOUS_RISK;
    if (eig_host[(size_t)b * o.m + o.m - 1] >= op->gamma[ik0 + b] * op->smin[ik0 + b]) f |= KC_KFLAG_SPURIOUS_RISK;
  }
  if (!allc) {
    kc::set_error("some k-points did not reach tol within maxit");
    return KC_ERR_NO_CONVERGENCE;
  }
  return KC_OK;
}

int kc_last_residual_history(const kc_op* op, int k, double* res_host, int* prec_host, int cap, int* count) {
  KC_ARG(op != nullptr && count != nullptr, "NULL op or count");
  KC_ARG(k >= 0 && (size_t)k < op->hist.size(), "k outside the last solve's k-points");
  const auto& h = op->hist[k];
  *count = (int)h.size();
  for (int i = 0; i < cap && (size_t)i < h.size(); ++i) {
    if (res_host) res_host[i] = h[i];
    if (prec_host) prec_host[i] = op->histp[k][i];
  }
  return KC_OK;
}

}  // extern "C"
