// Learned interpolation-point selector (an alternative to the QRCP selection of
// Sec. 2.1): per-grid-point descriptors of the occupied density, a
// 3 -> 64 -> 64 -> 1 SiLU network evaluated with bfloat16-rounded weights and
// FP32 arithmetic, the gradient of its weighted binary cross-entropy with
// deterministic block reductions, Adam, soft targets from a point set, greedy
// non-maximum-suppression selection, and the fit-residual probe that decides
// whether a proposed point set is kept or replaced by QRCP.
#include <cmath>

#include "common.h"

namespace exx {

namespace {

constexpr int HID = 64;
constexpr int NPARAM = HID * 3 + HID + HID * HID + HID + HID + 1;  // 4481
constexpr int OW1 = 0, OB1 = OW1 + HID * 3, OW2 = OB1 + HID, OB2 = OW2 + HID * HID,
              OW3 = OB2 + HID, OB3 = OW3 + HID;
constexpr int MNT = 256;

// round to nearest even at 8 significand bits (bfloat16); NaN stays NaN
__device__ __forceinline__ float bf16_round(float x) {
  if (x != x) return x;
  unsigned u = __float_as_uint(x);
  const unsigned lsb = (u >> 16) & 1u;
  u += 0x7fffu + lsb;
  return __uint_as_float(u & 0xffff0000u);
}

__device__ __forceinline__ float silu_f(float x) { return x / (1.0f + __expf(-x)); }
__device__ __forceinline__ float dsilu_f(float x) {
  const float s = 1.0f / (1.0f + __expf(-x));
  return s * (1.0f + x * (1.0f - s));
}

// stage the parameters in LDS; weights rounded to bfloat16, biases kept FP32
__device__ void stage_params(const float* __restrict__ theta, float* sp) {
  for (int e = threadIdx.x; e < NPARAM; e += blockDim.x) {
    const float v = theta[e];
    const bool bias = (e >= OB1 && e < OW2) || (e >= OB2 && e < OW3) || e == OB3;
    sp[e] = bias ? v : bf16_round(v);
  }
  __syncthreads();
}

// ---------------------------------------------------------------------------
// descriptors
// ---------------------------------------------------------------------------
constexpr int FEAT_NBLK = 1024;

// rho(r) = (1/N_k) sum |psi|^2 and the orbital-weight feature sum|psi|^4 / (sum|psi|^2)^2;
// per-block partial sums of rho for the mean
__global__ __launch_bounds__(MNT) void feat_density_kernel(const double2* __restrict__ psi,
                                                           long rows, long ng, int nk,
                                                           double* __restrict__ rho,
                                                           float* __restrict__ feat,
                                                           double* __restrict__ partial) {
  __shared__ double red[MNT];
  double acc = 0.0;
  for (long r = (long)blockIdx.x * MNT + threadIdx.x; r < ng; r += (long)gridDim.x * MNT) {
    double s2 = 0.0, s4 = 0.0;
    for (long w = 0; w < rows; ++w) {
      const double2 v = psi[w * ng + r];
      const double a = v.x * v.x + v.y * v.y;
      s2 += a;
      s4 += a * a;
    }
    const double rr = s2 / nk;
    rho[r] = rr;
    feat[r * 3 + 2] = (float)(s4 / fmax(s2 * s2, 1e-300));
    acc += rr;
  }
  red[threadIdx.x] = acc;
  __syncthreads();
  for (int k = MNT / 2; k > 0; k >>= 1) {
    if (threadIdx.x < k) red[threadIdx.x] += red[threadIdx.x + k];
    __syncthreads();
  }
  if (threadIdx.x == 0) partial[blockIdx.x] = red[0];
}

struct FeatArgs {
  int n[3];
  double h[3];
  double norm[6];
};

// log(rho / mean rho), log|grad rho| - (4/3) log rho (fourth-order periodic central
// differences), then standardisation of all three
__global__ __launch_bounds__(MNT) void feat_grad_kernel(const double* __restrict__ rho,
                                                        const double* __restrict__ partial,
                                                        float* __restrict__ feat, FeatArgs a) {
  __shared__ double s_mean;
  if (threadIdx.x == 0) {
    double s = 0.0;
    for (int b = 0; b < FEAT_NBLK; ++b) s += partial[b];
    s_mean = s / ((double)a.n[0] * a.n[1] * a.n[2]);
  }
  __syncthreads();
  const long ng = (long)a.n[0] * a.n[1] * a.n[2];
  const long r = (long)blockIdx.x * MNT + threadIdx.x;
  if (r >= ng) return;
  const int n23 = a.n[1] * a.n[2];
  const int g[3] = {(int)(r / n23), (int)((r / a.n[2]) % a.n[1]), (int)(r % a.n[2])};
  const int st[3] = {n23, a.n[2], 1};
  double g2 = 0.0;
  for (int ax = 0; ax < 3; ++ax) {
    double v[4];
    const int off[4] = {-2, -1, 1, 2};
    for (int t = 0; t < 4; ++t) {
      int c = (g[ax] + off[t]) % a.n[ax];
      if (c < 0) c += a.n[ax];
      v[t] = rho[r + (long)(c - g[ax]) * st[ax]];
    }
    const double d = (v[0] - 8.0 * v[1] + 8.0 * v[2] - v[3]) / (12.0 * a.h[ax]);
    g2 += d * d;
  }
  const double rr = rho[r];
  const double f0 = log(fmax(rr, 1e-300) / s_mean);
  const double f1 = 0.5 * log(fmax(g2, 1e-300)) - (4.0 / 3.0) * log(fmax(rr, 1e-300));
  const double f2 = feat[r * 3 + 2];
  feat[r * 3 + 0] = (float)((f0 - a.norm[0]) / a.norm[1]);
  feat[r * 3 + 1] = (float)((f1 - a.norm[2]) / a.norm[3]);
  feat[r * 3 + 2] = (float)((f2 - a.norm[4]) / a.norm[5]);
}

// ---------------------------------------------------------------------------
// network
// ---------------------------------------------------------------------------
__global__ __launch_bounds__(MNT) void mlp_forward_kernel(long n, const float* __restrict__ feat,
                                                          const float* __restrict__ theta,
                                                          float* __restrict__ score) {
  __shared__ float sp[NPARAM];
  stage_params(theta, sp);
  const long i = (long)blockIdx.x * MNT + threadIdx.x;
  if (i >= n) return;
  const float x0 = feat[i * 3], x1 = feat[i * 3 + 1], x2 = feat[i * 3 + 2];
  float h1[HID];
#pragma unroll
  for (int k = 0; k < HID; ++k)
    h1[k] = silu_f(sp[OW1 + 3 * k] * x0 + sp[OW1 + 3 * k + 1] * x1 + sp[OW1 + 3 * k + 2] * x2 +
                   sp[OB1 + k]);
  float s = sp[OB3];
  for (int j = 0; j < HID; ++j) {
    float z = sp[OB2 + j];
#pragma unroll
    for (int k = 0; k < HID; ++k) z += sp[OW2 + HID * j + k] * h1[k];
    s += sp[OW3 + j] * silu_f(z);
  }
  score[i] = s;
}

constexpr int BPTS = 64;     // points per pass of a workgroup in the gradient kernel
constexpr int GRAD_WG = 1024;  // at most this many workgroups (and partial rows)

// Per-workgroup partial gradient (not yet divided by the weight sum), weight
// sum and weighted loss sum. Workgroup b takes the point blocks b, b + G, b + 2G,
// ... (G workgroups, BPTS points per block) in that order, so the sums are
// deterministic. Point q of the batch is row idx[q] of feat / target (row q
// when idx is null); an index outside [0, rows) adds nothing.
__global__ __launch_bounds__(MNT) void mlp_grad_kernel(long n, const int32_t* __restrict__ idx,
                                                       long rows, const float* __restrict__ feat,
                                                       const float* __restrict__ tgt, float wpos,
                                                       const float* __restrict__ theta,
                                                       float* __restrict__ part) {
  __shared__ float sp[NPARAM];
  __shared__ float sh1[BPTS][HID + 1];
  __shared__ float sdz2[BPTS][HID + 1];
  __shared__ float sdz1[BPTS][HID + 1];
  __shared__ float sx[BPTS][3];
  __shared__ float sds[BPTS], sw[BPTS], sl[BPTS];
  stage_params(theta, sp);
  const int tid = threadIdx.x;
  // this workgroup's row of partial sums; entry e is only ever touched by thread e % MNT
  float* out = part + (long)blockIdx.x * (NPARAM + 2);
  for (int e = tid; e < NPARAM; e += MNT) out[e] = 0.f;
  float wsum = 0.f, lsum = 0.f;
  const long nblocks = (n + BPTS - 1) / BPTS;
  for (long pb = blockIdx.x; pb < nblocks; pb += gridDim.x) {
    // forward and backward of one point per thread of the first BPTS threads
    if (tid < BPTS) {
      const long q = pb * BPTS + tid;
      float ds = 0.f, w = 0.f, lo = 0.f;
      const long i = q < n ? (idx ? (long)idx[q] : q) : -1;
      if (i >= 0 && i < rows) {
        const float x0 = feat[i * 3], x1 = feat[i * 3 + 1], x2 = feat[i * 3 + 2];
        sx[tid][0] = x0;
        sx[tid][1] = x1;
        sx[tid][2] = x2;
        // z1 is parked in this point's row of sdz1, which later receives dL/dz1
        for (int k = 0; k < HID; ++k) {
          const float z1 = sp[OW1 + 3 * k] * x0 + sp[OW1 + 3 * k + 1] * x1 +
                           sp[OW1 + 3 * k + 2] * x2 + sp[OB1 + k];
          sdz1[tid][k] = z1;
          sh1[tid][k] = silu_f(z1);
        }
        float s = sp[OB3];
        for (int j = 0; j < HID; ++j) {
          float z = sp[OB2 + j];
#pragma unroll
          for (int k = 0; k < HID; ++k) z += sp[OW2 + HID * j + k] * sh1[tid][k];
          sdz2[tid][j] = z;  // holds z2 until the output gradient is known
          s += sp[OW3 + j] * silu_f(z);
        }
        const float t = tgt[i];
        w = 1.0f + wpos * t;
        const float sig = 1.0f / (1.0f + __expf(-s));
        ds = w * (sig - t);
        // softplus(s) - t s, in the overflow-free form
        lo = w * (fmaxf(s, 0.f) + log1pf(__expf(-fabsf(s))) - t * s);
#pragma unroll
        for (int j = 0; j < HID; ++j) sdz2[tid][j] = ds * sp[OW3 + j] * dsilu_f(sdz2[tid][j]);
        for (int k = 0; k < HID; ++k) {
          float dh = 0.f;
          for (int j = 0; j < HID; ++j) dh += sdz2[tid][j] * sp[OW2 + HID * j + k];
          sdz1[tid][k] = dh * dsilu_f(sdz1[tid][k]);
        }
      } else {
        for (int k = 0; k < HID; ++k) sh1[tid][k] = sdz2[tid][k] = sdz1[tid][k] = 0.f;
        sx[tid][0] = sx[tid][1] = sx[tid][2] = 0.f;
      }
      sds[tid] = ds;
      sw[tid] = w;
      sl[tid] = lo;
    }
    __syncthreads();
    // parameter gradients summed over the block's points
    for (int e = tid; e < NPARAM; e += MNT) {
      float sum = 0.f;
      if (e < OB1) {
        const int k = e / 3, c = e % 3;
        for (int p = 0; p < BPTS; ++p) sum += sdz1[p][k] * sx[p][c];
      } else if (e < OW2) {
        const int k = e - OB1;
        for (int p = 0; p < BPTS; ++p) sum += sdz1[p][k];
      } else if (e < OB2) {
        const int j = (e - OW2) / HID, k = (e - OW2) % HID;
        for (int p = 0; p < BPTS; ++p) sum += sdz2[p][j] * sh1[p][k];
      } else if (e < OW3) {
        const int j = e - OB2;
        for (int p = 0; p < BPTS; ++p) sum += sdz2[p][j];
      } else if (e < OB3) {
        // dL/dw3_j = ds h2_j, with h2_j = silu(z2_j) recomputed from h1
        const int j = e - OW3;
        for (int p = 0; p < BPTS; ++p) {
          if (sds[p] == 0.f) continue;
          float z = sp[OB2 + j];
          for (int k = 0; k < HID; ++k) z += sp[OW2 + HID * j + k] * sh1[p][k];
          sum += sds[p] * silu_f(z);
        }
      } else {
        for (int p = 0; p < BPTS; ++p) sum += sds[p];
      }
      out[e] += sum;
    }
    if (tid == 0) {
      for (int p = 0; p < BPTS; ++p) {
        wsum += sw[p];
        lsum += sl[p];
      }
    }
    __syncthreads();
  }
  if (tid == 0) {
    out[NPARAM] = wsum;
    out[NPARAM + 1] = lsum;
  }
}

// grad = (sum of partials) / (sum of weights), loss likewise; fixed summation order
__global__ __launch_bounds__(MNT) void mlp_grad_reduce_kernel(const float* __restrict__ part,
                                                              int nblk, float* __restrict__ grad,
                                                              double* __restrict__ loss) {
  const int e = blockIdx.x * MNT + threadIdx.x;
  if (e > NPARAM + 1) return;
  double s = 0.0, ws = 0.0;
  for (int b = 0; b < nblk; ++b) {
    s += (double)part[(long)b * (NPARAM + 2) + e];
    ws += (double)part[(long)b * (NPARAM + 2) + NPARAM];
  }
  if (e < NPARAM)
    grad[e] = (float)(s / ws);
  else if (e == NPARAM + 1)
    *loss = s / ws;
}

__global__ void adam_kernel(int np, float* __restrict__ theta, const float* __restrict__ g,
                            float* __restrict__ m, float* __restrict__ v, float lr, float b1,
                            float b2, float eps, float c1, float c2) {
  const int e = blockIdx.x * blockDim.x + threadIdx.x;
  if (e >= np) return;
  const float ge = g[e];
  const float me = b1 * m[e] + (1.f - b1) * ge;
  const float ve = b2 * v[e] + (1.f - b2) * ge * ge;
  m[e] = me;
  v[e] = ve;
  theta[e] -= lr * (me / c1) / (sqrtf(ve / c2) + eps);
}

// ---------------------------------------------------------------------------
// targets and NMS selection
// ---------------------------------------------------------------------------
struct GridArgs {
  int n[3];
  double L[3];
  double h;  // target width (targets) or suppression radius (NMS)
  int npts;
};

__device__ __forceinline__ double min_image_d2(const GridArgs& a, const double* x,
                                               const double* y) {
  double s = 0.0;
  for (int ax = 0; ax < 3; ++ax) {
    double d = x[ax] - y[ax];
    d -= a.L[ax] * rint(d / a.L[ax]);
    s += d * d;
  }
  return s;
}

__device__ __forceinline__ void coords(const GridArgs& a, long r, double* x) {
  const int n23 = a.n[1] * a.n[2];
  x[0] = (double)(r / n23) * (a.L[0] / a.n[0]);
  x[1] = (double)((r / a.n[2]) % a.n[1]) * (a.L[1] / a.n[1]);
  x[2] = (double)(r % a.n[2]) * (a.L[2] / a.n[2]);
}

__global__ __launch_bounds__(MNT) void targets_kernel(const int32_t* __restrict__ pts,
                                                      float* __restrict__ t, GridArgs a) {
  extern __shared__ double sq[];  // 3 * npts
  for (int e = threadIdx.x; e < a.npts; e += MNT) coords(a, pts[e], sq + 3 * e);
  __syncthreads();
  const long ng = (long)a.n[0] * a.n[1] * a.n[2];
  const long r = (long)blockIdx.x * MNT + threadIdx.x;
  if (r >= ng) return;
  double x[3];
  coords(a, r, x);
  double best = 1e300;
  for (int p = 0; p < a.npts; ++p) best = fmin(best, min_image_d2(a, x, sq + 3 * p));
  t[r] = (float)exp(-best / (2.0 * a.h * a.h));
}

constexpr int SEL_NT = 1024;

// order of candidates: higher score first, NaN after every number, ties to the
// smaller index; bi < 0 means "no candidate yet"
__device__ __forceinline__ bool nms_better(float v, long i, float bv, long bi) {
  if (bi < 0) return true;
  const bool vn = v != v, bn = bv != bv;
  if (vn != bn) return bn;
  if (vn) return i < bi;
  return (v > bv) || (v == bv && i < bi);
}

// better of (v, i) and (v2, i2) in nms_better order; i < 0 marks "none"
__device__ __forceinline__ void nms_take(float& v, int& i, float v2, int i2) {
  if (i2 >= 0 && (i < 0 || nms_better(v2, i2, v, i))) {
    v = v2;
    i = i2;
  }
}

__device__ __forceinline__ void nms_wave_reduce(float& v, int& i) {
#pragma unroll
  for (int off = 32; off > 0; off >>= 1) {
    const float v2 = __shfl_xor(v, off);
    const int i2 = __shfl_xor(i, off);
    nms_take(v, i, v2, i2);
  }
}

struct NmsBox {
  int k[3];  // half-width of the search box in grid steps per axis (0 = whole axis)
};

constexpr int NMS_WAVES = SEL_NT / 64;

// One workgroup: greedy selection by score, suppressing alive points closer
// than h to each pick; if nothing is alive before k picks, the remaining slots
// take the unpicked points in score order. The grid is cut into SEL_NT
// contiguous chunks whose best alive candidate sits in LDS; a pick only
// rescans the chunks whose best it suppressed, and suppression only visits the
// box of grid points within h along every axis (min-image distances are the
// ones of the full scan, so the result is that of the plain greedy rule).
// alive: [N_g] scratch (1 alive, 0 suppressed, 2 picked). k <= N_g.
__global__ __launch_bounds__(SEL_NT) void nms_kernel(const float* __restrict__ score,
                                                     int32_t* __restrict__ alive, int k,
                                                     int32_t* __restrict__ pts, GridArgs a,
                                                     NmsBox box) {
  const int ng = a.n[0] * a.n[1] * a.n[2];
  const int chunk = (ng + SEL_NT - 1) / SEL_NT;
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  __shared__ float sbv[SEL_NT];
  __shared__ int sbi[SEL_NT];
  __shared__ unsigned char dirty[SEL_NT];
  __shared__ int dlist[SEL_NT];
  __shared__ int ndirty;
  __shared__ float wv[NMS_WAVES];
  __shared__ int wi[NMS_WAVES];
  __shared__ int s_pick;
  for (int r = tid * chunk; r < min(ng, (tid + 1) * chunk); ++r) alive[r] = 1;
  dirty[tid] = 1;
  const double h2 = a.h * a.h;
  const double dx[3] = {a.L[0] / a.n[0], a.L[1] / a.n[1], a.L[2] / a.n[2]};
  int bx[3];
  for (int ax = 0; ax < 3; ++ax) bx[ax] = box.k[ax] > 0 ? 2 * box.k[ax] + 1 : a.n[ax];
  const int nbox = bx[0] * bx[1] * bx[2];
  int count = 0;
  __syncthreads();
  for (int pass = 0; pass < 2; ++pass) {  // pass 0: with suppression, pass 1: fill
    while (count < k) {
      // rescan dirty chunks, one wave per chunk
      if (tid == 0) ndirty = 0;
      __syncthreads();
      if (dirty[tid]) {
        dlist[atomicAdd(&ndirty, 1)] = tid;
        dirty[tid] = 0;
      }
      __syncthreads();
      for (int j = wave; j < ndirty; j += NMS_WAVES) {
        const int c = dlist[j];
        const int lo = c * chunk, hi = min(ng, lo + chunk);
        float v = 0.f;
        int bi = -1;
        for (int r = lo + lane; r < hi; r += 64)
          if (alive[r] == 1) nms_take(v, bi, score[r], r);
        nms_wave_reduce(v, bi);
        if (lane == 0) {
          sbv[c] = v;
          sbi[c] = bi;
        }
      }
      __syncthreads();
      // best alive point
      float v = sbv[tid];
      int bi = sbi[tid];
      nms_wave_reduce(v, bi);
      if (lane == 0) {
        wv[wave] = v;
        wi[wave] = bi;
      }
      __syncthreads();
      if (wave == 0) {
        v = lane < NMS_WAVES ? wv[lane] : 0.f;
        bi = lane < NMS_WAVES ? wi[lane] : -1;
        nms_wave_reduce(v, bi);
        if (lane == 0) s_pick = bi;
      }
      __syncthreads();
      const int pick = s_pick;
      if (pick < 0) break;  // nothing alive in this pass (uniform)
      if (tid == 0) {
        pts[count] = pick;
        alive[pick] = 2;
        dirty[pick / chunk] = 1;
      }
      if (pass == 0) {
        const int n23 = a.n[1] * a.n[2];
        const int pc[3] = {pick / n23, (pick / a.n[2]) % a.n[1], pick % a.n[2]};
        double cx[3];
        for (int ax = 0; ax < 3; ++ax) cx[ax] = (double)pc[ax] * dx[ax];
        for (int t = tid; t < nbox; t += SEL_NT) {
          const int o[3] = {t / (bx[1] * bx[2]), (t / bx[2]) % bx[1], t % bx[2]};
          int g[3];
          for (int ax = 0; ax < 3; ++ax) {
            if (box.k[ax] > 0) {
              g[ax] = (pc[ax] + o[ax] - box.k[ax]) % a.n[ax];
              if (g[ax] < 0) g[ax] += a.n[ax];
            } else {
              g[ax] = o[ax];
            }
          }
          const int r = (g[0] * a.n[1] + g[1]) * a.n[2] + g[2];
          if (alive[r] != 1) continue;
          double x[3];
          for (int ax = 0; ax < 3; ++ax) x[ax] = (double)g[ax] * dx[ax];
          if (min_image_d2(a, x, cx) < h2) {
            alive[r] = 0;
            const int c = r / chunk;
            if (sbi[c] == r) dirty[c] = 1;
          }
        }
      }
      __syncthreads();
      ++count;
    }
    // revive suppressed points for the fill pass
    for (int r = tid * chunk; r < min(ng, (tid + 1) * chunk); ++r)
      if (alive[r] == 0) alive[r] = 1;
    dirty[tid] = 1;
    __syncthreads();
  }
}

// ---------------------------------------------------------------------------
// fit-residual probe
// ---------------------------------------------------------------------------
// probe grid points from a counter-based generator (SplitMix64 of seed + j)
__global__ void probe_points_kernel(int nr, unsigned long long seed, long ng,
                                    int32_t* __restrict__ probe) {
  const int j = blockIdx.x * blockDim.x + threadIdx.x;
  if (j >= nr) return;
  unsigned long long z = seed + 0x9e3779b97f4a7c15ull * (unsigned long long)(j + 1);
  z = (z ^ (z >> 30)) * 0xbf58476d1ce4e5b9ull;
  z = (z ^ (z >> 27)) * 0x94d049bb133111ebull;
  z = z ^ (z >> 31);
  probe[j] = (int32_t)(z % (unsigned long long)ng);
}

// A[p][w] = psi[w][x_p], x = pts (p < np) then probe (p >= np); w over N_k n_occ rows
__global__ __launch_bounds__(MNT) void probe_gather_kernel(const double2* __restrict__ psi,
                                                           long ng, int rows,
                                                           const int32_t* __restrict__ pts, int np,
                                                           const int32_t* __restrict__ probe,
                                                           double2* __restrict__ A) {
  const int w = blockIdx.x * MNT + threadIdx.x;
  const int p = blockIdx.y;
  if (w >= rows) return;
  long x = p < np ? pts[p] : probe[p - np];
  x = x < 0 ? 0 : (x >= ng ? ng - 1 : x);  // caller indices are clamped into the grid
  A[(long)p * rows + w] = psi[(long)w * ng + x];
}

// Cpp[P][Q] = |G[P][Q]|^2, Cpr[P][r] = |G[P][np + r]|^2 (stored complex, zero imaginary)
__global__ __launch_bounds__(MNT) void probe_abs2_kernel(const double2* __restrict__ G, int np,
                                                         int nr, double2* __restrict__ Cpp,
                                                         double2* __restrict__ Cpr) {
  const long e = (long)blockIdx.x * MNT + threadIdx.x;
  const long nx = np + nr;
  if (e >= (long)np * nx) return;
  const int P = (int)(e / nx), c = (int)(e % nx);
  const double2 v = G[e];
  const double2 a = make_double2(v.x * v.x + v.y * v.y, 0.0);
  if (c < np)
    Cpp[(long)P * np + c] = a;
  else
    Cpr[(long)P * nr + (c - np)] = a;
}

// C(r, r) = (sum_w |psi_w(r)|^2)^2 for the probe rows of A
__global__ __launch_bounds__(MNT) void probe_diag_kernel(const double2* __restrict__ A, int rows,
                                                         int np, double* __restrict__ crr) {
  __shared__ double red[MNT];
  const double2* a = A + (long)(np + blockIdx.x) * rows;
  double s = 0.0;
  for (int w = threadIdx.x; w < rows; w += MNT) s += a[w].x * a[w].x + a[w].y * a[w].y;
  red[threadIdx.x] = s;
  __syncthreads();
  for (int k = MNT / 2; k > 0; k >>= 1) {
    if (threadIdx.x < k) red[threadIdx.x] += red[threadIdx.x + k];
    __syncthreads();
  }
  if (threadIdx.x == 0) crr[blockIdx.x] = red[0] * red[0];
}

// residual = sum_r max(C(r,r) - |W C(P,r)|^2, 0) / sum_r C(r,r), one workgroup
__global__ __launch_bounds__(1024) void probe_residual_kernel(const double2* __restrict__ Y,
                                                              const double* __restrict__ crr,
                                                              int np, int nr,
                                                              double* __restrict__ resid) {
  __shared__ double rn[1024], rd[1024];
  double num = 0.0, den = 0.0;
  for (int r = threadIdx.x; r < nr; r += 1024) {
    double q = 0.0;
    for (int P = 0; P < np; ++P) {
      const double2 y = Y[(long)P * nr + r];
      q += y.x * y.x + y.y * y.y;
    }
    num += fmax(crr[r] - q, 0.0);
    den += crr[r];
  }
  rn[threadIdx.x] = num;
  rd[threadIdx.x] = den;
  __syncthreads();
  for (int k = 512; k > 0; k >>= 1) {
    if (threadIdx.x < k) {
      rn[threadIdx.x] += rn[threadIdx.x + k];
      rd[threadIdx.x] += rd[threadIdx.x + k];
    }
    __syncthreads();
  }
  if (threadIdx.x == 0) *resid = rd[0] > 0.0 ? rn[0] / rd[0] : 1.0;
}

GridArgs grid_args(const Geom& g, int npts) {
  GridArgs a;
  for (int i = 0; i < 3; ++i) {
    a.n[i] = g.n[i];
    a.L[i] = g.L[i];
  }
  a.h = 0.5 * pow(g.omega / (double)npts, 1.0 / 3.0);
  a.npts = npts;
  return a;
}

size_t al256(size_t b) { return (b + 255) / 256 * 256; }

struct ProbeLayout {
  size_t probe, A, G, Cpp, Cpr, W, T, Y, keep, rank, tol, crr, total;
};

ProbeLayout probe_layout(const Geom& g, int nr) {
  const size_t np = (size_t)g.ni, rows = (size_t)g.nk * g.no, nx = np + nr;
  ProbeLayout L;
  size_t o = 0;
  auto take = [&](size_t bytes) {
    const size_t at = o;
    o += al256(bytes);
    return at;
  };
  L.probe = take(sizeof(int32_t) * nr);
  L.A = take(sizeof(double2) * nx * rows);
  L.G = take(sizeof(double2) * np * nx);
  L.Cpp = take(sizeof(double2) * np * np);
  L.Cpr = take(sizeof(double2) * np * nr);
  L.W = take(sizeof(double2) * np * np);
  L.T = take(sizeof(double2) * 32 * np);
  L.Y = take(sizeof(double2) * np * nr);
  L.keep = take(sizeof(int32_t) * np);
  L.rank = take(sizeof(int32_t));
  L.tol = take(sizeof(double));
  L.crr = take(sizeof(double) * nr);
  L.total = o;
  return L;
}

// column sums and sums of squares of feat [n][3] in FP64: block b sums the
// rows b, b + gridDim.x, ... (a fixed assignment), a fixed-order tree in LDS
constexpr int MOM_WG = 512;
__global__ __launch_bounds__(MNT) void mlp_moments_kernel(long n, const float* __restrict__ feat,
                                                         double* __restrict__ part) {
  __shared__ double red[6][MNT];
  double acc[6] = {0, 0, 0, 0, 0, 0};
  for (long i = (long)blockIdx.x * MNT + threadIdx.x; i < n; i += (long)gridDim.x * MNT) {
#pragma unroll
    for (int j = 0; j < 3; ++j) {
      const double f = (double)feat[3 * i + j];
      acc[j] += f;
      acc[3 + j] += f * f;
    }
  }
#pragma unroll
  for (int j = 0; j < 6; ++j) red[j][threadIdx.x] = acc[j];
  __syncthreads();
  for (int w = MNT / 2; w > 0; w >>= 1) {
    if ((int)threadIdx.x < w) {
#pragma unroll
      for (int j = 0; j < 6; ++j) red[j][threadIdx.x] += red[j][threadIdx.x + w];
    }
    __syncthreads();
  }
  if (threadIdx.x < 6) part[(long)blockIdx.x * 6 + threadIdx.x] = red[threadIdx.x][0];
}

// sums[j] += sum over the blocks' partial sums, in block order
__global__ void mlp_moments_reduce_kernel(const double* __restrict__ part, int nblk,
                                          double* __restrict__ sums) {
  const int j = threadIdx.x;
  if (j >= 6) return;
  double s = 0.0;
  for (int b = 0; b < nblk; ++b) s += part[(long)b * 6 + j];
  sums[j] += s;
}

}  // namespace

size_t mlp_feature_scratch_bytes(const Geom& g) {
  return al256(sizeof(double) * (size_t)g.ng) + sizeof(double) * FEAT_NBLK;
}

hipError_t launch_mlp_features(const Geom& g, const double2* psi, const double* norm, float* feat,
                               void* scratch, hipStream_t st) {
  double* rho = (double*)scratch;
  double* partial = (double*)((char*)scratch + al256(sizeof(double) * (size_t)g.ng));
  hipLaunchKernelGGL(feat_density_kernel, dim3(FEAT_NBLK), dim3(MNT), 0, st, psi,
                     (long)g.nk * g.no, (long)g.ng, g.nk, rho, feat, partial);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  FeatArgs a;
  for (int i = 0; i < 3; ++i) {
    a.n[i] = g.n[i];
    a.h[i] = g.L[i] / g.n[i];
  }
  for (int i = 0; i < 6; ++i) a.norm[i] = norm[i];
  hipLaunchKernelGGL(feat_grad_kernel, dim3((unsigned)((g.ng + MNT - 1) / MNT)), dim3(MNT), 0, st,
                     rho, partial, feat, a);
  return hipGetLastError();
}

hipError_t launch_mlp_forward(long n, const float* feat, const float* theta, float* score,
                              hipStream_t st) {
  if (n <= 0) return hipSuccess;
  hipLaunchKernelGGL(mlp_forward_kernel, dim3((unsigned)((n + MNT - 1) / MNT)), dim3(MNT), 0, st,
                     n, feat, theta, score);
  return hipGetLastError();
}

static int grad_workgroups(long n) {
  const long nb = (n + BPTS - 1) / BPTS;
  return (int)(nb < GRAD_WG ? nb : GRAD_WG);
}

size_t mlp_grad_scratch_bytes(long n) {
  return sizeof(float) * (size_t)grad_workgroups(n) * (NPARAM + 2);
}

hipError_t launch_mlp_grad(long n, const int32_t* idx, long rows, const float* feat,
                           const float* tgt, float wpos, const float* theta, float* grad,
                           double* loss, void* scratch, hipStream_t st) {
  const int nblk = grad_workgroups(n);
  hipLaunchKernelGGL(mlp_grad_kernel, dim3(nblk), dim3(MNT), 0, st, n, idx, rows, feat, tgt, wpos,
                     theta, (float*)scratch);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL(mlp_grad_reduce_kernel, dim3((NPARAM + 2 + MNT - 1) / MNT), dim3(MNT), 0, st,
                     (const float*)scratch, nblk, grad, loss);
  return hipGetLastError();
}

hipError_t launch_adam(int np, float* theta, const float* g, float* m, float* v, int step, float lr,
                       float b1, float b2, float eps, hipStream_t st) {
  const float c1 = 1.f - powf(b1, (float)step), c2 = 1.f - powf(b2, (float)step);
  hipLaunchKernelGGL(adam_kernel, dim3((np + 255) / 256), dim3(256), 0, st, np, theta, g, m, v, lr,
                     b1, b2, eps, c1, c2);
  return hipGetLastError();
}

hipError_t launch_targets(const Geom& g, const int32_t* pts, int npts, double sigma, float* t,
                          hipStream_t st) {
  GridArgs a = grid_args(g, npts);
  a.h = sigma;
  hipLaunchKernelGGL(targets_kernel, dim3((unsigned)((g.ng + MNT - 1) / MNT)), dim3(MNT),
                     sizeof(double) * 3 * npts, st, pts, t, a);
  return hipGetLastError();
}

size_t mlp_nms_scratch_bytes(const Geom& g) { return sizeof(int32_t) * (size_t)g.ng; }

hipError_t launch_nms(const Geom& g, const float* score, int k, int32_t* pts, void* scratch,
                      hipStream_t st) {
  GridArgs a = grid_args(g, k);
  // box half-widths: every point closer than h along an axis lies within
  // floor(h / spacing) + 1 steps; an axis the box would wrap around is taken whole
  NmsBox box;
  for (int ax = 0; ax < 3; ++ax) {
    const long kk = (long)floor(a.h / (g.L[ax] / g.n[ax])) + 1;
    box.k[ax] = (2 * kk + 1 >= g.n[ax]) ? 0 : (int)kk;
  }
  hipLaunchKernelGGL(nms_kernel, dim3(1), dim3(SEL_NT), 0, st, score, (int32_t*)scratch, k, pts, a,
                     box);
  return hipGetLastError();
}

size_t mlp_probe_scratch_bytes(const Geom& g, int nr) { return probe_layout(g, nr).total; }

hipError_t launch_mlp_probe(const Geom& g, const double2* psi, const int32_t* pts, int nr,
                            unsigned long long seed, double* resid, void* scratch,
                            hipStream_t st) {
  const ProbeLayout L = probe_layout(g, nr);
  char* ws = (char*)scratch;
  int32_t* probe = (int32_t*)(ws + L.probe);
  double2* A = (double2*)(ws + L.A);
  double2* G = (double2*)(ws + L.G);
  double2* Cpp = (double2*)(ws + L.Cpp);
  double2* Cpr = (double2*)(ws + L.Cpr);
  double2* W = (double2*)(ws + L.W);
  double2* Y = (double2*)(ws + L.Y);
  double* crr = (double*)(ws + L.crr);
  const int np = g.ni, rows = g.nk * g.no, nx = np + nr;
  hipLaunchKernelGGL(probe_points_kernel, dim3((nr + 255) / 256), dim3(256), 0, st, nr, seed,
                     (long)g.ng, probe);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL(probe_gather_kernel, dim3((rows + MNT - 1) / MNT, nx), dim3(MNT), 0, st, psi,
                     (long)g.ng, rows, pts, np, probe, A);
  if ((e = hipGetLastError()) != hipSuccess) return e;
  // Gram of the points against points and probes: G = A_P A^H
  e = gemm<double, double, double, double>(np, nx, rows, 1, A_N, A, rows, 0, B_C, A, rows, 0, G, nx,
                                           0, 1.0, false, st);
  if (e != hipSuccess) return e;
  const long ne = (long)np * nx;
  hipLaunchKernelGGL(probe_abs2_kernel, dim3((unsigned)((ne + MNT - 1) / MNT)), dim3(MNT), 0, st, G,
                     np, nr, Cpp, Cpr);
  if ((e = hipGetLastError()) != hipSuccess) return e;
  hipLaunchKernelGGL(probe_diag_kernel, dim3(nr), dim3(MNT), 0, st, A, rows, np, crr);
  if ((e = hipGetLastError()) != hipSuccess) return e;
  // C(P,P) = L L^H with the fit's pivot-drop rule, W = L^{-1}, Y = W C(P, probe)
  Geom gp = g;
  gp.nk = 1;
  e = launch_chol_blocked(gp, Cpp, (int32_t*)(ws + L.keep), (int32_t*)(ws + L.rank),
                          (double*)(ws + L.tol), 1e-12, st);
  if (e != hipSuccess) return e;
  e = launch_tri_inv_blocked(gp, Cpp, (const int32_t*)(ws + L.keep), W, (double2*)(ws + L.T), st);
  if (e != hipSuccess) return e;
  e = gemm<double, double, double, double>(np, nr, np, 1, A_N, W, np, 0, B_N, Cpr, nr, 0, Y, nr, 0,
                                           1.0, false, st);
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL(probe_residual_kernel, dim3(1), dim3(1024), 0, st, Y, crr, np, nr, resid);
  return hipGetLastError();
}

static int moment_workgroups(long n) {
  const long nb = (n + MNT - 1) / MNT;
  return (int)(nb < MOM_WG ? (nb < 1 ? 1 : nb) : MOM_WG);
}

size_t mlp_moments_scratch_bytes(long n) { return sizeof(double) * 6 * (size_t)moment_workgroups(n); }

hipError_t launch_mlp_moments(long n, const float* feat, double* sums, void* scratch,
                              hipStream_t st) {
  const int nblk = moment_workgroups(n);
  hipLaunchKernelGGL(mlp_moments_kernel, dim3(nblk), dim3(MNT), 0, st, n, feat, (double*)scratch);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL(mlp_moments_reduce_kernel, dim3(1), dim3(64), 0, st, (const double*)scratch,
                     nblk, sums);
  return hipGetLastError();
}

}  // namespace exx
