// Layout permutes and entry attribution.
#include <hip/hip_runtime.h>

#include "kernels.hpp"

namespace cq {

namespace {

struct PermArgs {
  const void* src;
  void* dst;
  int64_t total;
  int naxes;
  int log2[kMaxPermAxes];
  int64_t sstride[kMaxPermAxes];
  double alpha;
};

// Generic axis permutation with conversion: one destination element per
// thread iteration, destination written contiguously.
template <typename TS, typename TD>
__global__ void __launch_bounds__(256) permute_kernel(PermArgs p) {
  const TS* __restrict__ src = static_cast<const TS*>(p.src);
  TD* __restrict__ dst = static_cast<TD*>(p.dst);
  const int64_t step = (int64_t)gridDim.x * blockDim.x;
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < p.total; i += step) {
    int64_t r = i, off = 0;
    for (int a = p.naxes - 1; a >= 0; --a) {
      const int l = p.log2[a];
      off += (r & (((int64_t)1 << l) - 1)) * p.sstride[a];
      r >>= l;
    }
    dst[i] = TD(p.alpha * double(src[off]));
  }
}

// ---------------------------------------------------------------------------
// Attribution (Section 3.1).  Two separable passes, both FP64:
//  1. measured ends: U[j][lm][b] = sum_m prod_u sigma(lm_u, m_u)
//                                  * V[j][basis(lm)][compose(b, m)]
//  2. initialised ends: E[row(li, lm)][b] = sum_j prod_t alpha(li_t, j_t) U[j][lm][b]
// Thread per output element; b is the fastest index so stores are contiguous.
// ---------------------------------------------------------------------------

struct AttrArgs {
  const double* V;
  double* U;
  double* E;
  int r, o, n, w, k;
  int out_pos[CQ_MAX_WIDTH];
  int meas_pos[CQ_MAX_WIDTH];
  int64_t init_w[CQ_MAX_WIDTH];
  int64_t meas_w[CQ_MAX_WIDTH];
};

// Measurement basis of a label: I and Z -> Z basis (0), X -> 1, Y -> 2.
__device__ inline int basis_of(int l) { return l == 3 ? 0 : l; }

// alpha(label, prepared state) for states |0>, |1>, |+>, |+i> = 0..3; only
// called on the support (I, Z: |0>, |1>; X: also |+>; Y: also |+i>).
__device__ inline double alpha_coef(int l, int d) {
  if (d >= 2) return 2.0;
  if (l == 0) return 1.0;
  if (l == 3) return d == 0 ? 1.0 : -1.0;
  return -1.0;
}

__global__ void __launch_bounds__(256) attr_meas_kernel(AttrArgs a) {
  const int64_t nb = (int64_t)1 << a.n;
  const int64_t nlm = (int64_t)1 << (2 * a.o);
  const int64_t total = ((int64_t)1 << (2 * a.r)) * nlm * nb;
  int64_t pow3o = 1;
  for (int u = 0; u < a.o; ++u) pow3o *= 3;
  const int64_t step = (int64_t)gridDim.x * blockDim.x;
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < total; i += step) {
    const int64_t b = i % nb;
    const int64_t lm = (i / nb) % nlm;
    const int64_t j = i / (nb * nlm);
    int64_t x0 = 0;
    for (int q = 0; q < a.n; ++q)
      if ((b >> (a.n - 1 - q)) & 1) x0 |= (int64_t)1 << a.out_pos[q];
    int64_t beta = 0;
    for (int u = 0; u < a.o; ++u) beta = 3 * beta + basis_of((lm >> (2 * (a.o - 1 - u))) & 3);
    const double* Vj = a.V + ((j * pow3o + beta) << a.w);
    double sum = 0.0;
    for (int m = 0; m < (1 << a.o); ++m) {
      int64_t x = x0;
      bool neg = false;
      for (int u = 0; u < a.o; ++u) {
        if ((m >> (a.o - 1 - u)) & 1) {
          x |= (int64_t)1 << a.meas_pos[u];
          if (((lm >> (2 * (a.o - 1 - u))) & 3) != 0) neg = !neg;
        }
      }
      const double v = Vj[x];
      sum += neg ? -v : v;
    }
    a.U[i] = sum;
  }
}

__global__ void __launch_bounds__(256) attr_init_kernel(AttrArgs a) {
  const int64_t nb = (int64_t)1 << a.n;
  const int64_t nlm = (int64_t)1 << (2 * a.o);
  const int64_t nli = (int64_t)1 << (2 * a.r);
  const int64_t total = nli * nlm * nb;
  const int64_t step = (int64_t)gridDim.x * blockDim.x;
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < total; i += step) {
    const int64_t b = i % nb;
    const int64_t lm = (i / nb) % nlm;
    const int64_t li = i / (nb * nlm);
    // support of each init digit: I, Z -> {0, 1}; X -> {0, 1, 2}; Y -> {0, 1, 3}
    int64_t combos = 1;
    for (int t = 0; t < a.r; ++t) {
      const int l = (li >> (2 * (a.r - 1 - t))) & 3;
      combos *= (l == 1 || l == 2) ? 3 : 2;
    }
    double sum = 0.0;
    for (int64_t c = 0; c < combos; ++c) {
      int64_t rem = c, j = 0;
      double coef = 1.0;
      // mixed radix over the supports, last init slot fastest
      for (int t = a.r - 1; t >= 0; --t) {
        const int l = (li >> (2 * (a.r - 1 - t))) & 3;
        const int sz = (l == 1 || l == 2) ? 3 : 2;
        int d = (int)(rem % sz);
        rem /= sz;
        if (d == 2) d = (l == 1) ? 2 : 3;
        j += (int64_t)d << (2 * (a.r - 1 - t));
        coef *= alpha_coef(l, d);
      }
      sum += coef * a.U[(j * nlm + lm) * nb + b];
    }
    int64_t row = 0;
    for (int t = 0; t < a.r; ++t) row += ((li >> (2 * (a.r - 1 - t))) & 3) * a.init_w[t];
    for (int u = 0; u < a.o; ++u) row += ((lm >> (2 * (a.o - 1 - u))) & 3) * a.meas_w[u];
    a.E[row * nb + b] = sum;
  }
}

unsigned grid_for(int64_t total) {
  int64_t b = (total + 255) / 256;
  if (b > 1 << 20) b = 1 << 20;
  if (b < 1) b = 1;
  return (unsigned)b;
}

}  // namespace

hipError_t launch_permute(const PermLaunch& p, hipStream_t stream) {
  PermArgs a;
  a.src = p.src;
  a.dst = p.dst;
  a.naxes = p.naxes;
  int bits = 0;
  for (int i = 0; i < p.naxes; ++i) {
    a.log2[i] = p.log2[i];
    a.sstride[i] = p.sstride[i];
    bits += p.log2[i];
  }
  a.total = (int64_t)1 << bits;
  a.alpha = p.alpha;
  const unsigned grid = grid_for(a.total);
  const bool s64 = p.ts == DType::F64, d64 = p.td == DType::F64;
  if (s64 && d64) hipLaunchKernelGGL((permute_kernel<double, double>), dim3(grid), dim3(256), 0, stream, a);
  else if (s64) hipLaunchKernelGGL((permute_kernel<double, float>), dim3(grid), dim3(256), 0, stream, a);
  else if (d64) hipLaunchKernelGGL((permute_kernel<float, double>), dim3(grid), dim3(256), 0, stream, a);
  else hipLaunchKernelGGL((permute_kernel<float, float>), dim3(grid), dim3(256), 0, stream, a);
  return hipGetLastError();
}

hipError_t launch_attribute(const AttrLaunch& l, hipStream_t stream) {
  AttrArgs a;
  a.V = l.V;
  a.U = l.U;
  a.E = l.E;
  a.r = l.r;
  a.o = l.o;
  a.n = l.n;
  a.w = l.w;
  a.k = l.k;
  for (int i = 0; i < CQ_MAX_WIDTH; ++i) {
    a.out_pos[i] = l.out_pos[i];
    a.meas_pos[i] = l.meas_pos[i];
    a.init_w[i] = l.init_w[i];
    a.meas_w[i] = l.meas_w[i];
  }
  const int64_t total = ((int64_t)1 << (2 * (l.r + l.o))) << l.n;
  const unsigned grid = grid_for(total);
  hipLaunchKernelGGL(attr_meas_kernel, dim3(grid), dim3(256), 0, stream, a);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL(attr_init_kernel, dim3(grid), dim3(256), 0, stream, a);
  return hipGetLastError();
}

}  // namespace cq
