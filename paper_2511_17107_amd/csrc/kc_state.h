// Internal state of a kc_op handle and the launchers shared between translation units.
#pragma once

#include <vector>

#include "kc_common.h"

namespace kc {

// Largest number of materials (entries of the inverse-permittivity table).
constexpr int KC_MAX_MAT = 64;

// Operator and preconditioner passes whose tile width is tuned per handle.
enum TilePass { TP_X1 = 0, TP_Y1, TP_ZA, TP_ZB, TP_ZT, TP_Y2, TP_X2, TP_X1P, TP_ZF, TP_X2P, TP_NPASS };

// Inverse-permittivity entry of one material in compute precision T: the real diagonal
// (eps^-1)_cc and the upper off-diagonals (eps^-1)_12, _13, _23, all pre-multiplied by 1/N^3
// (the normalisation of the two unnormalised 3D DFTs around the permittivity step).
template <typename T>
struct EpsEntry {
  T d[3];
  cpx<T> o[3];
};

// Device memory source of a handle: the caller's allocator callbacks (kc_create), or hipMalloc /
// hipFree when none are given.
struct Allocator {
  kc_alloc_fn alloc = nullptr;
  kc_free_fn free = nullptr;
  void* ctx = nullptr;
};

// Device buffer that grows on demand (contents are not preserved when it grows).  Memory comes
// from `al` (nullptr: hipMalloc).
struct DevBuf {
  void* p = nullptr;
  size_t bytes = 0;
  const Allocator* al = nullptr;
  int ensure(size_t n);  // zero-fills newly allocated memory
  void release();
  ~DevBuf() { release(); }
  template <typename T>
  T* as() const {
    return static_cast<T*>(p);
  }
};

struct SolverWork;  // LOBPCG buffers (kc_solver.hip)
struct Net;         // learned preconditioner (kc_nn.hip)

// Addressing of the vectors of a block operation: vector v belongs to k-point v / vpk and is
// column v % vpk of that k-point's group, stored at (v / vpk) * kstride + v % vpk (in units of
// one 3N^3 vector).  active[v] == 0 skips the vector (its output is left untouched).
struct VecMap {
  int vpk = 1;
  int kstride = 1;
  const int* active = nullptr;
  __host__ __device__ size_t off(int v) const { return (size_t)(v / vpk) * kstride + (v % vpk); }
  __device__ bool on(int v) const { return active == nullptr || active[v] != 0; }
};

}  // namespace kc

struct kc_op {
  int N = 0;
  int scheme = 0;
  int n_mat = 0;
  bool zoff = true;              // some material has (eps^-1)_13 or (eps^-1)_23 != 0
  int stencil_m = 1;             // order 2m of the curl/divergence stencils (eq (2.34))
  kc::Skew skew;                 // lattice transform of the symbols (eq (2.12)); cubic: l1d == nullptr
  kc::DevBuf lam1;               // Lambda_1(q): c64 [N] then c32 [N] (non-cubic lattices)
  kc::Allocator alloc;           // source of every device buffer of the handle
  int flags = 0;                 // KC_FLAG_* found by kc_create
  std::vector<double> smin;      // [nk] smallest positive s(p) = |K(p)|^2 (spurious-mode bound)
  std::vector<double> smax;      // [nk] largest s(p) (scale of the operator's rounding)
  std::vector<int> kflags;       // [nk] KC_KFLAG_* of each k-point
  std::vector<double> eps_host;  // [n_mat][3][3][2]
  double epsinv_norm = 1.0;      // largest absolute row sum of eps^-1 over the materials present
  kc::DevBuf ids;                // uint32 [N^3]: x-edge | y-edge << 8 | z-edge << 16 | vol << 24
  kc::DevBuf eps64, eps32;       // EpsEntry<double/float> [n_mat]
  kc::DevBuf tw64, tw32;         // twiddles exp(+2 pi i t/N), t < N
  int nk = 0;
  std::vector<double> kvec, gamma;  // [nk][3], [nk]
  kc::DevBuf ktab64, ktab32;        // 1D symbols [nk][3][N]
  std::vector<kc::c64> ktab_host;   // the same (FP64) on the host
  std::vector<kc::c64> lam1_host;   // Lambda_1(q) [N] on the host (non-cubic lattices)
  kc::DevBuf gamma_d;               // double [nk]
  kc::DevBuf sfloor_d;              // double [nk] floor of |K|^2 in the solver's preconditioners
  kc::DevBuf dcl_d;                 // int [nk] 1: the solver deflates the DC longitudinal direction
  std::vector<int> dcl;             // the same on the host
  kc::DevBuf work_a, work_b, work_c;  // operator intermediates
  kc::DevBuf work_k;                  // K . x per point (first x-pass -> last x-pass)
  kc::SolverWork* solver = nullptr;
  kc::Net* net = nullptr;     // attached learned preconditioner (not owned)
  kc::DevBuf epsfeat;         // f32 [N^3][9] inverse-permittivity features for the network
  kc::DevBuf efield;          // f32 [3][N^3] E_c = 1/(eps^-1)_cc at the c-edge points
  kc::DevBuf efield_t;        // the same, x-major ([3][x][z][y]) for the yz-plane pass
  kc::DevBuf efield_k;        // f32 [nb][3][N^3] learned fields of the k-points being solved
  kc::DevBuf efield_kt;       // the same, x-major ([nb][3][x][z][y]), written with efield_k
  kc::DevBuf kdev;            // double [nk][3] wave vectors
  kc::DevBuf train_buf;       // work vectors of kc_pcg, kc_perturbed_residuals, kc_net_loss_grad
  double stats[8] = {0, 0, 0, 0, 0, 0, 0, 0};
  std::vector<std::vector<double>> hist;  // per k-point of the last kc_solve: max Res_j per iteration
  std::vector<std::vector<int8_t>> histp; // ... and the precision of that iteration's AW
  int hist_ik0 = 0;
  int8_t tiles[2][16] = {};     // tile width per pass (kc::TilePass), [FP32, FP64]; 0 = default
  bool tuned[2] = {false, false};
  // every device buffer of the handle takes its memory from `alloc`
  void bind_allocator() {
    kc::DevBuf* bufs[] = {&ids, &eps64, &eps32, &tw64, &tw32, &ktab64, &ktab32, &gamma_d, &sfloor_d, &dcl_d, &lam1, &work_a, &work_b,
                          &work_c, &work_k, &epsfeat, &efield, &efield_t, &efield_k, &efield_kt, &kdev, &train_buf};
    for (kc::DevBuf* b : bufs) b->al = &alloc;
  }
};

namespace kc {

// y = Op x (kc_apply without argument checks); vectors v use k-point ik0 + v / vm.vpk.  With
// ev != nullptr, events ev[0..6] are recorded around the passes (6 passes for CrossDoF, 5 else).
int apply_op(kc_op* op, int ik0, int nvec, const VecMap& vm, const c64* x, c64* y, int prec,
             hipStream_t s, hipEvent_t* ev = nullptr);
// z = K_P^{-1} r
int apply_precond(kc_op* op, int ik0, int nvec, int vecs_per_k, const c64* r, c64* z,
                  hipStream_t s);
// y = T_E x, the transverse-projection preconditioner with the positive diagonal field E
// (f32 [3][N^3] per k-point group at field + (v / vm.vpk) * fkstride * 3N^3); x is addressed
// through vm, y through vmy (same grouping and active mask); x and y must not overlap.  sfl
// (device double per k-point of the call, or nullptr): floor of s = |K|^2 in the gains 1/s.
int apply_tp(kc_op* op, int ik0, int nvec, const VecMap& vm, const VecMap& vmy, const c64* x, c64* y,
             const float* field, int fkstride, int prec, hipStream_t s, const double* sfl = nullptr);
// per-grid kernel attributes (the LDS limit of the yz-plane pass); called by kc_create
int prepare_kernels(int N);
// E_c = 1/(eps^-1)_cc at the c-edge points (built on first use)
int build_efield(kc_op* op);
// g[b][3][N^3] += gradient with respect to E of sum_j w_j Re<e_j, T_E r_j> (w device, nvec
// values; vectors grouped vpk per k-point; FP64 transforms)
int tp_grad(kc_op* op, int ik0, int nvec, int vpk, const c64* r, const c64* e, const double* w, float* g,
            hipStream_t s);

}  // namespace kc
