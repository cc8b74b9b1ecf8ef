// Interpolation-point selection: greedy pivoted Cholesky of the pair Gram
// matrix |Gamma(r, r')|^2 (QR with column pivoting of the stacked occupied-pair
// matrix), FP64. One pivot per host-loop step, no host synchronisation: a
// device-side state records when pivoting stops, after which the remaining
// slots are filled by descending density.
#include "common.h"

namespace exx {

namespace {

constexpr int SNT = 256;
constexpr int SNB = 512;  // blocks of the argmax pass

struct SelState {
  int done;
  int npiv;
  int piv;
  int pad;
  double first;
  double dp;
};

struct SelBufs {
  double* dens;
  double* d;
  int32_t* taken;
  double* Lc;   // [n_isdf][N_g]
  double2* gv;  // [rows] conj psi(row, piv)
  double* pval;
  int32_t* pidx;
  SelState* st;
};

__device__ __forceinline__ bool better(double v, int i, double bv, int bi) {
  return (v > bv) || (v == bv && i < bi);
}

__global__ __launch_bounds__(SNT) void sel_init_kernel(const double2* __restrict__ psi, long rows,
                                                       long ng, SelBufs b) {
  const long r = (long)blockIdx.x * SNT + threadIdx.x;
  if (r == 0) {
    b.st->done = 0;
    b.st->npiv = 0;
    b.st->piv = -1;
    b.st->first = 0.0;
    b.st->dp = 0.0;
  }
  if (r >= ng) return;
  double s = 0.0;
  for (long w = 0; w < rows; ++w) {
    const double2 v = psi[w * ng + r];
    s += v.x * v.x + v.y * v.y;
  }
  b.dens[r] = s;
  b.d[r] = s * s;
  b.taken[r] = 0;
}

__device__ void block_argmax(double& bv, int& bi) {
  __shared__ double sv[SNT];
  __shared__ int si[SNT];
  sv[threadIdx.x] = bv;
  si[threadIdx.x] = bi;
  __syncthreads();
  for (int k = SNT / 2; k > 0; k >>= 1) {
    if (threadIdx.x < k) {
      if (better(sv[threadIdx.x + k], si[threadIdx.x + k], sv[threadIdx.x], si[threadIdx.x])) {
        sv[threadIdx.x] = sv[threadIdx.x + k];
        si[threadIdx.x] = si[threadIdx.x + k];
      }
    }
    __syncthreads();
  }
  bv = sv[0];
  bi = si[0];
  __syncthreads();
}

__global__ __launch_bounds__(SNT) void sel_argmax_kernel(long ng, SelBufs b) {
  const double* key = b.st->done ? b.dens : b.d;
  double bv = -1.0e300;
  int bi = 0x7fffffff;
  for (long r = (long)blockIdx.x * SNT + threadIdx.x; r < ng; r += (long)gridDim.x * SNT) {
    if (b.taken[r]) continue;
    const double v = key[r];
    if (better(v, (int)r, bv, bi)) {
      bv = v;
      bi = (int)r;
    }
  }
  block_argmax(bv, bi);
  if (threadIdx.x == 0) {
    b.pval[blockIdx.x] = bv;
    b.pidx[blockIdx.x] = bi;
  }
}

// decide slot p: a pivot (Schur diagonal still above tolerance) or a density fill
__global__ __launch_bounds__(SNT) void sel_decide_kernel(const double2* __restrict__ psi, long rows,
                                                         long ng, int p, double rel_tol,
                                                         int32_t* __restrict__ pts, SelBufs b) {
  double bv = -1.0e300;
  int bi = 0x7fffffff;
  for (int k = threadIdx.x; k < SNB; k += SNT) {
    if (better(b.pval[k], b.pidx[k], bv, bi)) {
      bv = b.pval[k];
      bi = b.pidx[k];
    }
  }
  block_argmax(bv, bi);
  __shared__ int s_mode;  // 0 pivot, 1 fill from the argmax above, 2 fill needs a rescan
  if (threadIdx.x == 0) {
    if (b.st->done) {
      s_mode = 1;
    } else {
      if (p == 0) b.st->first = bv;
      if (bv > rel_tol * b.st->first) {
        s_mode = 0;
      } else {
        b.st->done = 1;
        s_mode = 2;
      }
    }
  }
  __syncthreads();
  const int mode = s_mode;
  if (mode == 2) {
    bv = -1.0e300;
    bi = 0x7fffffff;
    for (long r = threadIdx.x; r < ng; r += SNT) {
      if (b.taken[r]) continue;
      const double v = b.dens[r];
      if (better(v, (int)r, bv, bi)) {
        bv = v;
        bi = (int)r;
      }
    }
    block_argmax(bv, bi);
  }
  if (threadIdx.x == 0) {
    pts[p] = bi;
    b.taken[bi] = 1;
    if (mode == 0) {
      b.st->piv = bi;
      b.st->dp = bv;
      b.st->npiv += 1;
    }
  }
  if (mode == 0) {
    for (long w = threadIdx.x; w < rows; w += SNT) {
      const double2 v = psi[w * ng + bi];
      b.gv[w] = make_double2(v.x, -v.y);
    }
  }
}

// column p of the Cholesky factor and the Schur-diagonal update
__global__ __launch_bounds__(SNT) void sel_update_kernel(const double2* __restrict__ psi, long rows,
                                                         long ng, int p, SelBufs b) {
  if (b.st->done) return;
  const long r = (long)blockIdx.x * SNT + threadIdx.x;
  if (r >= ng) return;
  const int piv = b.st->piv;
  double gx = 0.0, gy = 0.0;
  for (long w = 0; w < rows; ++w) {
    const double2 v = psi[w * ng + r];
    const double2 c = b.gv[w];
    gx += v.x * c.x - v.y * c.y;
    gy += v.x * c.y + v.y * c.x;
  }
  double col = gx * gx + gy * gy;
  for (int j = 0; j < p; ++j) col -= b.Lc[(long)j * ng + r] * b.Lc[(long)j * ng + piv];
  const double l = col / sqrt(b.st->dp);
  b.Lc[(long)p * ng + r] = l;
  b.d[r] -= l * l;
}

__global__ void sel_finish_kernel(SelBufs b, int32_t* n_pivot) { *n_pivot = b.st->npiv; }

SelBufs carve(const Geom& g, void* scratch) {
  char* c = (char*)scratch;
  auto take = [&](size_t bytes) {
    char* r = c;
    c += (bytes + 255) / 256 * 256;
    return r;
  };
  SelBufs b;
  const long rows = (long)g.nk * g.no;
  b.dens = (double*)take(sizeof(double) * g.ng);
  b.d = (double*)take(sizeof(double) * g.ng);
  b.taken = (int32_t*)take(sizeof(int32_t) * g.ng);
  b.Lc = (double*)take(sizeof(double) * (size_t)g.ni * g.ng);
  b.gv = (double2*)take(sizeof(double2) * rows);
  b.pval = (double*)take(sizeof(double) * SNB);
  b.pidx = (int32_t*)take(sizeof(int32_t) * SNB);
  b.st = (SelState*)take(sizeof(SelState));
  return b;
}

}  // namespace

size_t select_scratch_bytes(const Geom& g) {
  const long rows = (long)g.nk * g.no;
  size_t s = 0;
  auto add = [&](size_t bytes) { s += (bytes + 255) / 256 * 256; };
  add(sizeof(double) * g.ng);
  add(sizeof(double) * g.ng);
  add(sizeof(int32_t) * g.ng);
  add(sizeof(double) * (size_t)g.ni * g.ng);
  add(sizeof(double2) * rows);
  add(sizeof(double) * SNB);
  add(sizeof(int32_t) * SNB);
  add(sizeof(SelState));
  return s;
}

hipError_t launch_select(const Geom& g, const double2* psi, int32_t* pts, int32_t* n_pivot,
                         void* scratch, hipStream_t st) {
  SelBufs b = carve(g, scratch);
  const long rows = (long)g.nk * g.no;
  const long ng = g.ng;
  const unsigned nb = (unsigned)((ng + SNT - 1) / SNT);
  hipLaunchKernelGGL(sel_init_kernel, dim3(nb), dim3(SNT), 0, st, psi, rows, ng, b);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  for (int p = 0; p < g.ni; ++p) {
    hipLaunchKernelGGL(sel_argmax_kernel, dim3(SNB), dim3(SNT), 0, st, ng, b);
    hipLaunchKernelGGL(sel_decide_kernel, dim3(1), dim3(SNT), 0, st, psi, rows, ng, p, 1e-12, pts,
                       b);
    hipLaunchKernelGGL(sel_update_kernel, dim3(nb), dim3(SNT), 0, st, psi, rows, ng, p, b);
    e = hipGetLastError();
    if (e != hipSuccess) return e;
  }
  hipLaunchKernelGGL(sel_finish_kernel, dim3(1), dim3(1), 0, st, b, n_pivot);
  return hipGetLastError();
}

}  // namespace exx
