// Learned preconditioner: a three-layer periodic 3D convolution network (3x3x3 kernels,
// 32 hidden channels, leaky ReLU) that maps the dielectric structure around each cell (and the
// wave vector) to the positive diagonal field E of the transverse-projection preconditioner
// T_E (kc_op.hip): E_c = E0_c exp(clamp(net_c, -3, 3)) with E0_c = 1/(eps^-1)_cc at the c-edge
// points, so an untrained (near-zero) network gives the classical choice E0.  The network runs
// once per k-point and solve; every LOBPCG iteration then applies the linear, Hermitian
// positive semi-definite T_E.
//
// Numerics: BF16 weights and activations, FP32 accumulation on v_mfma_f32_16x16x16_bf16
// (implicit GEMM: M = output channels, N = 16 positions along x, K = 27 taps x input channels),
// FP32 master weights, FP32 weight gradients, Adam in FP32.
//
// Layouts: activations channels-last [batch][z][y][x][C] (C padded to a multiple of 16,
// padding channels zero); weights for the forward pass [co][tap][ci] (tap = (dz*3+dy)*3+dx,
// input offset d-1, circular), for the backward data pass [ci][26-tap][co].
#include <algorithm>
#include <cmath>
#include <cstring>
#include <random>
#include <vector>

#include "kc_nn.h"

namespace kc {

typedef short s4 __attribute__((ext_vector_type(4)));
typedef float f4 __attribute__((ext_vector_type(4)));

__device__ __forceinline__ uint16_t f2bf(float f) {
  uint32_t u = __float_as_uint(f);
  u += 0x7FFFu + ((u >> 16) & 1u);  // round to nearest, ties to even
  return (uint16_t)(u >> 16);
}
__device__ __forceinline__ float bf2f(uint16_t h) { return __uint_as_float((uint32_t)h << 16); }

static uint16_t f2bf_host(float f) {
  uint32_t u;
  std::memcpy(&u, &f, 4);
  u += 0x7FFFu + ((u >> 16) & 1u);
  return (uint16_t)(u >> 16);
}

constexpr float SLOPE = 0.01f;
// v_mfma_f32_16x16x16_bf16: lane l supplies A[l%16][4(l/16)+t] and B[4(l/16)+t][l%16]
// (t = 0..3) and holds D[4(l/16)+r][l%16], r = 0..3.
#define KC_BF16_ROW(g, r) (4 * (g) + (r))

// ------------------------------------------------------------------------------------
// conv3d on a tile of 16 x-positions x 4 y-rows at one z; wave w owns row w.
// MODE 0: y = leaky(conv + b) -> bf16      MODE 1: y = conv + b -> f32
// MODE 2: y = conv * (mask > 0 ? 1 : slope) -> bf16   (backward data through the activation)
// ------------------------------------------------------------------------------------
template <int CIP, int COP, int MODE>
__global__ __launch_bounds__(256) void k_conv3d(const uint16_t* __restrict__ X, const uint16_t* __restrict__ Wt,
                                                const float* __restrict__ bias, void* __restrict__ Y,
                                                const uint16_t* __restrict__ mask, int N) {
  constexpr int CL = CIP + 4;            // LDS channel stride (bf16), padded against conflicts
  constexpr int WL = 27 * CIP + 4;       // LDS weight row stride (bf16)
  __shared__ __align__(16) uint16_t xs[3 * 6 * 18 * CL];
  __shared__ __align__(16) uint16_t ws[COP * WL];
  const int nxt = N / 16, nyt = N / 4;
  unsigned bid = blockIdx.x;
  const int xt = bid % nxt;
  bid /= nxt;
  const int yt = bid % nyt;
  const int z = bid / nyt;
  const int bat = blockIdx.y;
  const size_t N3 = (size_t)N * N * N;
  const uint16_t* Xb = X + (size_t)bat * N3 * CIP;
  const int x0 = xt * 16, y0 = yt * 4;
  // weights
  for (int e = threadIdx.x; e < COP * 27 * CIP / 4; e += 256) {
    const int co = (e * 4) / (27 * CIP), rest = (e * 4) % (27 * CIP);
    *(uint2*)&ws[co * WL + rest] = *(const uint2*)&Wt[(size_t)e * 4];
  }
  // input halo: planes z-1..z+1, rows y0-1..y0+4, columns x0-1..x0+16 (circular)
  constexpr int CH4 = CIP / 4;
  for (int e = threadIdx.x; e < 3 * 6 * 18 * CH4; e += 256) {
    const int c4 = e % CH4;
    int p = e / CH4;
    const int hx = p % 18;
    p /= 18;
    const int hy = p % 6;
    const int hz = p / 6;
    const int gx = (x0 + hx - 1 + N) % N, gy = (y0 + hy - 1 + N) % N, gz = (z + hz - 1 + N) % N;
    const size_t pos = ((size_t)gz * N + gy) * N + gx;
    *(uint2*)&xs[((hz * 6 + hy) * 18 + hx) * CL + c4 * 4] = *(const uint2*)&Xb[pos * CIP + c4 * 4];
  }
  __syncthreads();
  const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
  const int j = lane & 15, g = lane >> 4;
  f4 acc[COP / 16];
#pragma unroll
  for (int mt = 0; mt < COP / 16; ++mt) acc[mt] = f4{0.f, 0.f, 0.f, 0.f};
  for (int dz = 0; dz < 3; ++dz)
    for (int dy = 0; dy < 3; ++dy)
#pragma unroll
      for (int dx = 0; dx < 3; ++dx) {
        const int tap = (dz * 3 + dy) * 3 + dx;
        const uint16_t* xrow = &xs[((dz * 6 + wave + dy) * 18 + j + dx) * CL];
#pragma unroll
        for (int cb = 0; cb < CIP / 16; ++cb) {
          const s4 bv = *(const s4*)&xrow[cb * 16 + 4 * g];
#pragma unroll
          for (int mt = 0; mt < COP / 16; ++mt) {
            const s4 av = *(const s4*)&ws[(mt * 16 + j) * WL + tap * CIP + cb * 16 + 4 * g];
            acc[mt] = __builtin_amdgcn_mfma_f32_16x16x16bf16_1k(av, bv, acc[mt], 0, 0, 0);
          }
        }
      }
  const size_t pos = ((size_t)z * N + y0 + wave) * N + x0 + j;
#pragma unroll
  for (int mt = 0; mt < COP / 16; ++mt)
#pragma unroll
    for (int r = 0; r < 4; ++r) {
      const int co = mt * 16 + KC_BF16_ROW(g, r);
      float v = acc[mt][r];
      if (MODE == 0) {
        v += bias[co];
        v = v > 0.f ? v : SLOPE * v;
        ((uint16_t*)Y)[((size_t)bat * N3 + pos) * COP + co] = f2bf(v);
      } else if (MODE == 1) {
        v += bias[co];
        ((float*)Y)[((size_t)bat * N3 + pos) * COP + co] = v;
      } else {
        const float h = bf2f(mask[((size_t)bat * N3 + pos) * COP + co]);
        v = h > 0.f ? v : SLOPE * v;
        ((uint16_t*)Y)[((size_t)bat * N3 + pos) * COP + co] = f2bf(v);
      }
    }
}

// ------------------------------------------------------------------------------------
// weight gradient: gW[co][tap][ci] = sum_pos gZ[pos][co] X[pos + off(tap)][ci],
// gb[co] = sum_pos gZ[pos][co]; partials per block (FP32), then a fixed-order reduction.
// Block = 256 threads; thread t owns (co, ci) pairs t, t+256, ... of COP x CIP.
// ------------------------------------------------------------------------------------
template <int CIP, int COP>
__global__ __launch_bounds__(256) void k_conv3d_wgrad(const uint16_t* __restrict__ X, const uint16_t* __restrict__ GZ,
                                                      float* __restrict__ part, int N, int batch,
                                                      int tiles_per_block) {
  constexpr int CL = CIP + 4;
  constexpr int NPAIR = COP * CIP;
  constexpr int PPT = (NPAIR + 255) / 256;
  __shared__ __align__(16) uint16_t xs[3 * 6 * 18 * CL];
  __shared__ float gz[64 * COP];
  float acc[PPT][27];
  float bacc = 0.f;
#pragma unroll
  for (int q = 0; q < PPT; ++q)
#pragma unroll
    for (int t = 0; t < 27; ++t) acc[q][t] = 0.f;
  const int nxt = N / 16, nyt = N / 4;
  const size_t N3 = (size_t)N * N * N;
  const long ntile = (long)nxt * nyt * N * batch;
  for (long tile = (long)blockIdx.x * tiles_per_block;
       tile < std::min(ntile, (long)(blockIdx.x + 1) * tiles_per_block); ++tile) {
    long b2 = tile;
    const int xt = b2 % nxt;
    b2 /= nxt;
    const int yt = b2 % nyt;
    b2 /= nyt;
    const int z = b2 % N;
    const int bat = (int)(b2 / N);
    const int x0 = xt * 16, y0 = yt * 4;
    const uint16_t* Xb = X + (size_t)bat * N3 * CIP;
    __syncthreads();
    for (int e = threadIdx.x; e < 3 * 6 * 18 * (CIP / 4); e += 256) {
      const int c4 = e % (CIP / 4);
      int p = e / (CIP / 4);
      const int hx = p % 18;
      p /= 18;
      const int hy = p % 6;
      const int hz = p / 6;
      const int gx = (x0 + hx - 1 + N) % N, gy = (y0 + hy - 1 + N) % N, gzz = (z + hz - 1 + N) % N;
      const size_t pos = ((size_t)gzz * N + gy) * N + gx;
      *(uint2*)&xs[((hz * 6 + hy) * 18 + hx) * CL + c4 * 4] = *(const uint2*)&Xb[pos * CIP + c4 * 4];
    }
    for (int e = threadIdx.x; e < 64 * COP; e += 256) {
      const int co = e % COP, p = e / COP;
      const int px = p % 16, py = p / 16;
      const size_t pos = ((size_t)z * N + y0 + py) * N + x0 + px;
      gz[p * COP + co] = bf2f(GZ[((size_t)bat * N3 + pos) * COP + co]);
    }
    __syncthreads();
#pragma unroll
    for (int q = 0; q < PPT; ++q) {
      const int pr = threadIdx.x + q * 256;
      if (pr >= NPAIR) continue;
      const int co = pr / CIP, ci = pr % CIP;
      for (int p = 0; p < 64; ++p) {
        const float gv = gz[p * COP + co];
        const int px = p % 16, py = p / 16;
#pragma unroll
        for (int t = 0; t < 27; ++t) {
          const int dz = t / 9, dy = (t / 3) % 3, dx = t % 3;
          acc[q][t] += gv * bf2f(xs[((dz * 6 + py + dy) * 18 + px + dx) * CL + ci]);
        }
      }
    }
    if (threadIdx.x < COP) {
      for (int p = 0; p < 64; ++p) bacc += gz[p * COP + threadIdx.x];
    }
  }
  float* out = part + (size_t)blockIdx.x * (COP * 27 * CIP + COP);
#pragma unroll
  for (int q = 0; q < PPT; ++q) {
    const int pr = threadIdx.x + q * 256;
    if (pr >= NPAIR) continue;
    const int co = pr / CIP, ci = pr % CIP;
#pragma unroll
    for (int t = 0; t < 27; ++t) out[(co * 27 + t) * CIP + ci] = acc[q][t];
  }
  if (threadIdx.x < COP) out[COP * 27 * CIP + threadIdx.x] = bacc;
}

__global__ void k_sum_parts(const float* __restrict__ part, int nblk, int len, float* __restrict__ out) {
  const int e = blockIdx.x * blockDim.x + threadIdx.x;
  if (e >= len) return;
  float s = 0.f;
  for (int b = 0; b < nblk; ++b) s += part[(size_t)b * len + e];
  out[e] = s;
}

// MSE: g = 2 (y - t) / count (as bf16 for the backward passes), loss partial sums
__global__ void k_mse(const float* __restrict__ y, const float* __restrict__ t, uint16_t* __restrict__ g,
                      size_t count, float inv_count, double* __restrict__ part) {
  __shared__ double sh[256];
  double s = 0.0;
  for (size_t e = (size_t)blockIdx.x * 256 + threadIdx.x; e < count; e += (size_t)gridDim.x * 256) {
    const float d = y[e] - t[e];
    s += (double)d * d;
    g[e] = f2bf(2.f * d * inv_count);
  }
  sh[threadIdx.x] = s;
  __syncthreads();
  for (int o = 128; o > 0; o >>= 1) {
    if ((int)threadIdx.x < o) sh[threadIdx.x] += sh[threadIdx.x + o];
    __syncthreads();
  }
  if (threadIdx.x == 0) part[blockIdx.x] = sh[0];
}

// output gradient given directly (f32 -> bf16 for the backward passes)
__global__ void k_to_bf16(const float* __restrict__ g, uint16_t* __restrict__ o, size_t count) {
  for (size_t e = (size_t)blockIdx.x * 256 + threadIdx.x; e < count; e += (size_t)gridDim.x * 256)
    o[e] = f2bf(g[e]);
}

// Adam (Kingma & Ba) on FP32 master parameters
__global__ void k_adam(float* __restrict__ p, const float* __restrict__ g, float* __restrict__ m,
                       float* __restrict__ v, size_t n, float lr, float b1, float b2, float eps, float c1,
                       float c2) {
  for (size_t e = (size_t)blockIdx.x * 256 + threadIdx.x; e < n; e += (size_t)gridDim.x * 256) {
    const float gg = g[e];
    const float mm = b1 * m[e] + (1.f - b1) * gg;
    const float vv = b2 * v[e] + (1.f - b2) * gg * gg;
    m[e] = mm;
    v[e] = vv;
    p[e] -= lr * (mm / c1) / (sqrtf(vv / c2) + eps);
  }
}

// Master layout of one layer: W[co][ci][27] then b[co] (unpadded co x ci).  Packed: forward
// Wt[co][tap][ci] (COP x 27 x CIP, zero padding), backward Wb[ci][26 - tap][co] (CIP x 27 x COP).
__global__ void k_pack(const float* __restrict__ W, int co_n, int ci_n, int CIP, int COP,
                       uint16_t* __restrict__ Wt, uint16_t* __restrict__ Wb, float* __restrict__ bpad,
                       const float* __restrict__ b) {
  const int e = blockIdx.x * blockDim.x + threadIdx.x;
  if (e < COP * 27 * CIP) {
    const int co = e / (27 * CIP), rest = e % (27 * CIP), tap = rest / CIP, ci = rest % CIP;
    const float v = (co < co_n && ci < ci_n) ? W[((size_t)co * ci_n + ci) * 27 + tap] : 0.f;
    Wt[e] = f2bf(v);
    Wb[((size_t)ci * 27 + (26 - tap)) * COP + co] = f2bf(v);
  }
  if (e < COP) bpad[e] = (e < co_n) ? b[e] : 0.f;
}

// gradient of padded packed -> master layout
__global__ void k_unpack_grad(const float* __restrict__ gpad, int co_n, int ci_n, int CIP, int COP,
                              float* __restrict__ gW, float* __restrict__ gb) {
  const int e = blockIdx.x * blockDim.x + threadIdx.x;
  if (e < co_n * ci_n * 27) {
    const int co = e / (ci_n * 27), rest = e % (ci_n * 27), ci = rest / 27, tap = rest % 27;
    gW[e] = gpad[((size_t)co * 27 + tap) * CIP + ci];
  }
  if (e < co_n) gb[e] = gpad[(size_t)COP * 27 * CIP + e];
}

// ------------------------------------------------------------------------------------
// features (structure -> network) and the learned field (network -> T_E)
// ------------------------------------------------------------------------------------
// bf16 [nk][N3][32] per k-point: inverse-permittivity features (9), log E0 (3), k/pi (3), zeros.
__global__ void k_features(const float* __restrict__ epsf, const float* __restrict__ e0,
                           const double* __restrict__ kv, int N, int nk, uint16_t* __restrict__ F) {
  const size_t N3 = (size_t)N * N * N;
  for (size_t t = (size_t)blockIdx.x * 256 + threadIdx.x; t < N3 * nk; t += (size_t)gridDim.x * 256) {
    const size_t b = t / N3, p = t - b * N3;
    const double* k = kv + 3 * b;
    uint16_t* o = F + t * 32;
    float ch[32];
#pragma unroll
    for (int c = 0; c < 9; ++c) ch[c] = epsf[p * 9 + c];
#pragma unroll
    for (int c = 0; c < 3; ++c) ch[9 + c] = logf(e0[c * N3 + p]);
#pragma unroll
    for (int c = 0; c < 3; ++c) ch[12 + c] = (float)(k[c] * 0.31830988618379067);
#pragma unroll
    for (int c = 15; c < 32; ++c) ch[c] = 0.f;
#pragma unroll
    for (int c = 0; c < 32; c += 4) {
      uint2 w;
      w.x = (uint32_t)f2bf(ch[c]) | ((uint32_t)f2bf(ch[c + 1]) << 16);
      w.y = (uint32_t)f2bf(ch[c + 2]) | ((uint32_t)f2bf(ch[c + 3]) << 16);
      *(uint2*)&o[c] = w;
    }
  }
}

// E[b][c][p] = E0[c][p] exp(clamp(y[b][p][c], -3, 3)) from the network output y (f32 [nk][N3][16])
__global__ void k_efield(const float* __restrict__ y, const float* __restrict__ e0, int N, int nk,
                         float* __restrict__ E, float* __restrict__ Et) {
  const size_t N3 = (size_t)N * N * N;
  for (size_t t = (size_t)blockIdx.x * 256 + threadIdx.x; t < N3 * nk; t += (size_t)gridDim.x * 256) {
    const size_t b = t / N3, p = t - b * N3;
    const size_t xm = Et ? ((p % N) * N + p / ((size_t)N * N)) * N + (p / N) % N : 0;  // [x][z][y]
#pragma unroll
    for (int c = 0; c < 3; ++c) {
      const float o = fminf(fmaxf(y[t * 16 + c], -3.f), 3.f);
      const float e = e0[c * N3 + p] * expf(o);
      E[(b * 3 + c) * N3 + p] = e;
      if (Et) Et[(b * 3 + c) * N3 + xm] = e;
    }
  }
}

// ------------------------------------------------------------------------------------
// host side
// ------------------------------------------------------------------------------------
static const int LAYER_CI[3] = {NN_CIN, NN_CH, NN_CH};
static const int LAYER_CO[3] = {NN_CH, NN_CH, NN_COUT};
static const int LAYER_CIP[3] = {32, 32, 32};
static const int LAYER_COP[3] = {32, 32, 16};

size_t nn_param_count() {
  size_t s = 0;
  for (int l = 0; l < 3; ++l) s += (size_t)LAYER_CO[l] * LAYER_CI[l] * 27 + LAYER_CO[l];
  return s;
}

static size_t layer_offset(int l) {
  size_t s = 0;
  for (int i = 0; i < l; ++i) s += (size_t)LAYER_CO[i] * LAYER_CI[i] * 27 + LAYER_CO[i];
  return s;
}

int nn_init(Net* net, uint64_t seed) {
  const size_t np = nn_param_count();
  std::vector<float> p(np, 0.f);
  std::mt19937_64 rng(seed);
  for (int l = 0; l < 3; ++l) {
    const size_t off = layer_offset(l);
    const int fan_in = LAYER_CI[l] * 27;
    // He-normal for the hidden layers; the last layer starts near zero so that the learned
    // field starts as E0
    const double sd = (l < 2) ? std::sqrt(2.0 / fan_in) : 1e-3 / std::sqrt((double)fan_in);
    std::normal_distribution<double> nd(0.0, sd);
    for (size_t i = 0; i < (size_t)LAYER_CO[l] * LAYER_CI[l] * 27; ++i) p[off + i] = (float)nd(rng);
  }
  KC_TRY(net->params.ensure(np * sizeof(float)));
  KC_TRY(net->grads.ensure(np * sizeof(float)));
  KC_TRY(net->adam_m.ensure(np * sizeof(float)));
  KC_TRY(net->adam_v.ensure(np * sizeof(float)));
  for (int l = 0; l < 3; ++l) {
    KC_TRY(net->wt[l].ensure((size_t)LAYER_COP[l] * 27 * LAYER_CIP[l] * 2));
    KC_TRY(net->wb[l].ensure((size_t)LAYER_CIP[l] * 27 * LAYER_COP[l] * 2));
    KC_TRY(net->bpad[l].ensure((size_t)LAYER_COP[l] * 4));
  }
  KC_HIP(hipMemcpy(net->params.p, p.data(), np * sizeof(float), hipMemcpyHostToDevice));
  net->step = 0;
  return nn_pack(net, nullptr);
}

int nn_pack(Net* net, hipStream_t s) {
  const float* P = net->params.as<float>();
  for (int l = 0; l < 3; ++l) {
    const size_t off = layer_offset(l);
    const int n = LAYER_COP[l] * 27 * LAYER_CIP[l];
    k_pack<<<(n + 255) / 256, 256, 0, s>>>(P + off, LAYER_CO[l], LAYER_CI[l], LAYER_CIP[l], LAYER_COP[l],
                                            net->wt[l].as<uint16_t>(), net->wb[l].as<uint16_t>(),
                                            net->bpad[l].as<float>(),
                                            P + off + (size_t)LAYER_CO[l] * LAYER_CI[l] * 27);
    KC_LAUNCHED();
  }
  return KC_OK;
}

template <int CIP, int COP, int MODE>
static int conv(const uint16_t* X, const uint16_t* W, const float* b, void* Y, const uint16_t* mask, int N, int batch,
                hipStream_t s) {
  dim3 grid((N / 16) * (N / 4) * N, batch);
  k_conv3d<CIP, COP, MODE><<<grid, 256, 0, s>>>(X, W, b, Y, mask, N);
  KC_LAUNCHED();
  return KC_OK;
}

int nn_forward(Net* net, int N, int batch, const uint16_t* in, float* out, hipStream_t s) {
  if (N % 16 != 0) {
    set_error("learned preconditioner needs N divisible by 16");
    return KC_ERR_UNSUPPORTED;
  }
  const size_t N3 = (size_t)N * N * N;
  KC_TRY(net->h1.ensure((size_t)batch * N3 * 32 * 2));
  KC_TRY(net->h2.ensure((size_t)batch * N3 * 32 * 2));
  uint16_t* h1 = net->h1.as<uint16_t>();
  uint16_t* h2 = net->h2.as<uint16_t>();
  KC_TRY((conv<32, 32, 0>(in, net->wt[0].as<uint16_t>(), net->bpad[0].as<float>(), h1, nullptr, N, batch, s)));
  KC_TRY((conv<32, 32, 0>(h1, net->wt[1].as<uint16_t>(), net->bpad[1].as<float>(), h2, nullptr, N, batch, s)));
  KC_TRY((conv<32, 16, 1>(h2, net->wt[2].as<uint16_t>(), net->bpad[2].as<float>(), out, nullptr, N, batch, s)));
  return KC_OK;
}

template <int CIP, int COP>
static int wgrad(const uint16_t* X, const uint16_t* GZ, int N, int batch, DevBuf& part, float* out, hipStream_t s) {
  const long ntile = (long)(N / 16) * (N / 4) * N * batch;
  const int nblk = (int)std::min<long>(ntile, 512);
  const int tpb = (int)((ntile + nblk - 1) / nblk);
  const int len = COP * 27 * CIP + COP;
  KC_TRY(part.ensure((size_t)nblk * len * sizeof(float)));
  k_conv3d_wgrad<CIP, COP><<<nblk, 256, 0, s>>>(X, GZ, part.as<float>(), N, batch, tpb);
  KC_LAUNCHED();
  k_sum_parts<<<(len + 255) / 256, 256, 0, s>>>(part.as<float>(), nblk, len, out);
  KC_LAUNCHED();
  return KC_OK;
}

// backward pass from the bf16 output gradient in net->g3 (forward activations in h1, h2)
static int nn_backward_g3(Net* net, int N, int batch, const uint16_t* in, hipStream_t s) {
  const size_t N3 = (size_t)N * N * N;
  KC_TRY(net->g2.ensure((size_t)batch * N3 * 32 * 2));
  KC_TRY(net->g1.ensure((size_t)batch * N3 * 32 * 2));
  uint16_t* g3 = net->g3.as<uint16_t>();
  uint16_t* g2 = net->g2.as<uint16_t>();
  uint16_t* g1 = net->g1.as<uint16_t>();
  // backward data: gz2 = (W3^T * g3) masked by h2; gz1 = (W2^T * gz2) masked by h1
  KC_TRY((conv<16, 32, 2>(g3, net->wb[2].as<uint16_t>(), nullptr, g2, net->h2.as<uint16_t>(), N, batch, s)));
  KC_TRY((conv<32, 32, 2>(g2, net->wb[1].as<uint16_t>(), nullptr, g1, net->h1.as<uint16_t>(), N, batch, s)));
  // weight gradients (padded layout) -> master layout
  KC_TRY(net->gpad.ensure((size_t)(32 * 27 * 32 + 32) * 4));
  float* G = net->grads.as<float>();
  const uint16_t* xin[3] = {in, net->h1.as<uint16_t>(), net->h2.as<uint16_t>()};
  const uint16_t* gz[3] = {g1, g2, g3};
  for (int l = 0; l < 3; ++l) {
    if (LAYER_COP[l] == 32) {
      KC_TRY((wgrad<32, 32>(xin[l], gz[l], N, batch, net->wpart, net->gpad.as<float>(), s)));
    } else {
      KC_TRY((wgrad<32, 16>(xin[l], gz[l], N, batch, net->wpart, net->gpad.as<float>(), s)));
    }
    const size_t off = layer_offset(l);
    const int n = LAYER_CO[l] * LAYER_CI[l] * 27;
    k_unpack_grad<<<(n + 255) / 256, 256, 0, s>>>(net->gpad.as<float>(), LAYER_CO[l], LAYER_CI[l], LAYER_CIP[l],
                                                   LAYER_COP[l], G + off, G + off + n);
    KC_LAUNCHED();
  }
  return KC_OK;
}

int nn_gradients(Net* net, int N, int batch, const uint16_t* in, const float* target, double* loss_host,
                 hipStream_t s) {
  const size_t N3 = (size_t)N * N * N;
  KC_TRY(net->out.ensure((size_t)batch * N3 * 16 * 4));
  float* y = net->out.as<float>();
  KC_TRY(nn_forward(net, N, batch, in, y, s));
  KC_TRY(net->g3.ensure((size_t)batch * N3 * 16 * 2));
  const size_t count = (size_t)batch * N3 * 16;
  const int nb = (int)std::min<size_t>((count + 255) / 256, 1024);
  KC_TRY(net->lpart.ensure(nb * sizeof(double)));
  // loss over the used output channels: the padding channels of y and target are zero
  k_mse<<<nb, 256, 0, s>>>(y, target, net->g3.as<uint16_t>(), count, 1.f / (float)((size_t)batch * N3 * NN_COUT),
                           net->lpart.as<double>());
  KC_LAUNCHED();
  KC_TRY(nn_backward_g3(net, N, batch, in, s));
  if (loss_host) {
    std::vector<double> lp(nb);
    KC_HIP(hipMemcpyAsync(lp.data(), net->lpart.p, nb * sizeof(double), hipMemcpyDeviceToHost, s));
    KC_HIP(hipStreamSynchronize(s));
    double L = 0.0;
    for (double v : lp) L += v;
    *loss_host = L / (double)((size_t)batch * N3 * NN_COUT);
  }
  return KC_OK;
}

int nn_backward(Net* net, int N, int batch, const uint16_t* in, const float* gout, hipStream_t s) {
  const size_t N3 = (size_t)N * N * N;
  KC_TRY(net->out.ensure((size_t)batch * N3 * 16 * 4));
  KC_TRY(nn_forward(net, N, batch, in, net->out.as<float>(), s));
  KC_TRY(net->g3.ensure((size_t)batch * N3 * 16 * 2));
  const size_t count = (size_t)batch * N3 * 16;
  k_to_bf16<<<(unsigned)std::min<size_t>((count + 255) / 256, 4096), 256, 0, s>>>(gout, net->g3.as<uint16_t>(),
                                                                                  count);
  KC_LAUNCHED();
  return nn_backward_g3(net, N, batch, in, s);
}

int nn_adam(Net* net, float lr, float b1, float b2, float eps, hipStream_t s) {
  const size_t np = nn_param_count();
  net->step += 1;
  const float c1 = 1.f - std::pow(b1, (float)net->step), c2 = 1.f - std::pow(b2, (float)net->step);
  k_adam<<<(unsigned)std::min<size_t>((np + 255) / 256, 1024), 256, 0, s>>>(
      net->params.as<float>(), net->grads.as<float>(), net->adam_m.as<float>(), net->adam_v.as<float>(), np, lr,
      b1, b2, eps, c1, c2);
  KC_LAUNCHED();
  return nn_pack(net, s);
}

// network input of k-points ik0..ik0+nk-1 (bf16 [nk][N3][32])
int nn_features(kc_op* op, int ik0, int nk, uint16_t* F, hipStream_t s) {
  const int N = op->N;
  const size_t N3 = (size_t)N * N * N;
  if (op->epsfeat.p == nullptr) KC_TRY(nn_build_eps_features(op));
  KC_TRY(build_efield(op));
  const unsigned g = (unsigned)std::min<size_t>((N3 * nk + 255) / 256, 65535);
  k_features<<<g, 256, 0, s>>>(op->epsfeat.as<float>(), op->efield.as<float>(), op->kdev.as<double>() + 3 * (size_t)ik0,
                               N, nk, F);
  KC_LAUNCHED();
  return KC_OK;
}

// learned fields E of k-points ik0..ik0+nk-1 (f32 [nk][3][N3]) with the attached network
int nn_efield(kc_op* op, int ik0, int nk, float* E, hipStream_t s, float* Et) {
  Net* net = op->net;
  const int N = op->N;
  const size_t N3 = (size_t)N * N * N;
  KC_TRY(net->feat.ensure((size_t)nk * N3 * 32 * 2));
  KC_TRY(net->out.ensure((size_t)nk * N3 * 16 * 4));
  KC_TRY(nn_features(op, ik0, nk, net->feat.as<uint16_t>(), s));
  KC_TRY(nn_forward(net, N, nk, net->feat.as<uint16_t>(), net->out.as<float>(), s));
  const unsigned g = (unsigned)std::min<size_t>((N3 * nk + 255) / 256, 65535);
  k_efield<<<g, 256, 0, s>>>(net->out.as<float>(), op->efield.as<float>(), N, nk, E, Et);
  KC_LAUNCHED();
  return KC_OK;
}

int learned_fields(kc_op* op, int ik0, int nk, hipStream_t s) {
  const size_t bytes = (size_t)nk * 3 * op->N * op->N * op->N * sizeof(float);
  KC_TRY(op->efield_k.ensure(bytes));
  KC_TRY(op->efield_kt.ensure(bytes));
  return nn_efield(op, ik0, nk, op->efield_k.as<float>(), s, op->efield_kt.as<float>());
}

// E0_c = 1/(eps^-1)_cc of the material at the c-edge points (f32 [3][N3])
int build_efield(kc_op* op) {
  if (op->efield.p != nullptr) return KC_OK;
  const int N = op->N;
  const size_t N3 = (size_t)N * N * N;
  std::vector<uint32_t> ids(N3);
  KC_HIP(hipMemcpy(ids.data(), op->ids.p, N3 * 4, hipMemcpyDeviceToHost));
  std::vector<float> f(3 * N3);
  const double* t = op->eps_host.data();
  for (size_t p = 0; p < N3; ++p)
    for (int c = 0; c < 3; ++c) {
      const int m = (ids[p] >> (8 * c)) & 255;
      f[c * N3 + p] = (float)(1.0 / t[((m * 3 + c) * 3 + c) * 2]);
    }
  std::vector<float> ft(3 * N3);  // x-major copy: [c][x][z][y]
  for (int c = 0; c < 3; ++c)
    for (int z = 0; z < N; ++z)
      for (int y = 0; y < N; ++y)
        for (int x = 0; x < N; ++x)
          ft[c * N3 + ((size_t)x * N + z) * N + y] = f[c * N3 + ((size_t)z * N + y) * N + x];
  KC_TRY(op->efield_t.ensure(ft.size() * sizeof(float)));
  KC_HIP(hipMemcpy(op->efield_t.p, ft.data(), ft.size() * sizeof(float), hipMemcpyHostToDevice));
  KC_TRY(op->efield.ensure(f.size() * sizeof(float)));
  KC_HIP(hipMemcpy(op->efield.p, f.data(), f.size() * sizeof(float), hipMemcpyHostToDevice));
  return KC_OK;
}

// inverse-permittivity features per cell (f32 [N3][9]): diagonal at the three edge points,
// Re/Im of the three upper off-diagonals at the volume point (unscaled table)
int nn_build_eps_features(kc_op* op) {
  const int N = op->N;
  const size_t N3 = (size_t)N * N * N;
  std::vector<uint32_t> ids(N3);
  KC_HIP(hipMemcpy(ids.data(), op->ids.p, N3 * 4, hipMemcpyDeviceToHost));
  std::vector<float> f(N3 * 9);
  const double* t = op->eps_host.data();
  auto E = [&](int m, int r, int c, int part) { return t[((m * 3 + r) * 3 + c) * 2 + part]; };
  for (size_t p = 0; p < N3; ++p) {
    const uint32_t w = ids[p];
    const int mx = w & 255, my = (w >> 8) & 255, mz = (w >> 16) & 255, mv = w >> 24;
    float* o = &f[p * 9];
    o[0] = (float)E(mx, 0, 0, 0);
    o[1] = (float)E(my, 1, 1, 0);
    o[2] = (float)E(mz, 2, 2, 0);
    o[3] = (float)E(mv, 0, 1, 0);
    o[4] = (float)E(mv, 0, 1, 1);
    o[5] = (float)E(mv, 0, 2, 0);
    o[6] = (float)E(mv, 0, 2, 1);
    o[7] = (float)E(mv, 1, 2, 0);
    o[8] = (float)E(mv, 1, 2, 1);
  }
  KC_TRY(op->epsfeat.ensure(f.size() * sizeof(float)));
  KC_HIP(hipMemcpy(op->epsfeat.p, f.data(), f.size() * sizeof(float), hipMemcpyHostToDevice));
  return KC_OK;
}

}  // namespace kc
