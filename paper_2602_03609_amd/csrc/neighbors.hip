// Correlation-based neighbor selection (Sec. "Correlation-based Vecchia neighbor
// selection", Alg. 2 semantics): exact top-m earlier points per query under a
// FP64 log-correlation key, ties to the lower index.
//
// Design (gfx950): the points of each integer time (a "slab") are bucketed in a
// uniform spatial grid shared by all slabs and stored contiguously (CSR built on
// the device: count, scan, scatter). One wavefront serves one query. Slabs are
// visited in increasing lag; within a slab, cells are visited in Chebyshev rings
// around the query's cell. Two exact bounds stop the scan: the lag bound (no
// candidate of a later slab can beat the current m-th key) and the ring bound
// (a candidate outside the rings visited so far lies at least d away, and the
// key is monotone in the distance; d carries a slack far above rounding error).
// Keys of 64 candidates are evaluated per step from coalesced loads; candidates
// beating the m-th entry are found with a ballot and either inserted one at a
// time into a sorted list held one entry per lane, or, when many, sorted across
// the wave (bitonic) and merged with the list.
#include <limits.h>
#include <math.h>

#include "internal.hpp"

namespace vif {

namespace {

__global__ void validate_times_kernel(int64_t n, const double* __restrict__ t,
                                      uint32_t* __restrict__ flag) {
  int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  double ti = t[i];
  uint32_t bits = 0;
  if (!isfinite(ti)) bits |= 1u;
  else if (ti != rint(ti)) bits |= 2u;
  if (i > 0 && !(ti >= t[i - 1])) bits |= 4u;
  if (bits) atomicOr(flag, bits);
}

// ---- bounding box and grid index ---------------------------------------------
constexpr int kRedBlocks = 256;

__global__ __launch_bounds__(256) void bbox_stage1(int64_t n, const double* __restrict__ sx,
                                                   const double* __restrict__ sy,
                                                   double* __restrict__ part) {
  __shared__ double sh[4][256];
  double v[4] = {INFINITY, -INFINITY, INFINITY, -INFINITY};
  for (int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x; i < n; i += (int64_t)kRedBlocks * 256) {
    const double x = sx[i], y = sy[i];
    v[0] = fmin(v[0], x);
    v[1] = fmax(v[1], x);
    v[2] = fmin(v[2], y);
    v[3] = fmax(v[3], y);
  }
#pragma unroll
  for (int c = 0; c < 4; ++c) sh[c][threadIdx.x] = v[c];
  __syncthreads();
  for (int st = 128; st > 0; st >>= 1) {
    if (threadIdx.x < st) {
      sh[0][threadIdx.x] = fmin(sh[0][threadIdx.x], sh[0][threadIdx.x + st]);
      sh[1][threadIdx.x] = fmax(sh[1][threadIdx.x], sh[1][threadIdx.x + st]);
      sh[2][threadIdx.x] = fmin(sh[2][threadIdx.x], sh[2][threadIdx.x + st]);
      sh[3][threadIdx.x] = fmax(sh[3][threadIdx.x], sh[3][threadIdx.x + st]);
    }
    __syncthreads();
  }
  if (threadIdx.x < 4) part[threadIdx.x * kRedBlocks + blockIdx.x] = sh[threadIdx.x][0];
}

__global__ __launch_bounds__(256) void bbox_stage2(const double* __restrict__ part,
                                                   double* __restrict__ out) {
  if (threadIdx.x < 4) {
    const int c = threadIdx.x;
    double r = part[c * kRedBlocks];
    for (int b = 1; b < kRedBlocks; ++b) {
      const double v = part[c * kRedBlocks + b];
      r = (c & 1) ? fmax(r, v) : fmin(r, v);
    }
    out[c] = r;
  }
}

__device__ __forceinline__ int cell_of(double v, double lo, double inv, int g) {
  int c = (int)((v - lo) * inv);
  return c < 0 ? 0 : (c >= g ? g - 1 : c);
}

__global__ void fill_i32_kernel(int32_t* __restrict__ p, int64_t cnt) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < cnt) p[i] = 0;
}

__global__ void grid_count_kernel(int64_t n, const double* __restrict__ sx,
                                  const double* __restrict__ sy, const double* __restrict__ t,
                                  double t0, GridArgs G, int32_t* __restrict__ counts,
                                  int32_t* __restrict__ key) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  const int slab = G.nslab > 1 ? min((int)((t[i] - t0) * G.islab), G.nslab - 1) : 0;
  const int cx = cell_of(sx[i], G.xmin, G.icw, G.gx);
  const int cy = cell_of(sy[i], G.ymin, G.ich, G.gy);
  int cell;
  if (G.morton) {
    cell = 0;
    for (int b = 0; b < 16; ++b) cell |= (((cx >> b) & 1) << (2 * b)) | (((cy >> b) & 1) << (2 * b + 1));
  } else {
    cell = cy * G.gx + cx;
  }
  const int k = slab * G.ncell + cell;
  key[i] = k;
  atomicAdd(&counts[k], 1);
}

// Exclusive scan of counts[0..len) into counts (in place), tile of 1024.
__global__ __launch_bounds__(1024) void scan_tiles_kernel(int32_t* __restrict__ a, int64_t len,
                                                          int32_t* __restrict__ bsum) {
  __shared__ int32_t sh[1024];
  const int64_t i = (int64_t)blockIdx.x * 1024 + threadIdx.x;
  const int32_t v = i < len ? a[i] : 0;
  sh[threadIdx.x] = v;
  __syncthreads();
  for (int off = 1; off < 1024; off <<= 1) {
    const int32_t add = threadIdx.x >= off ? sh[threadIdx.x - off] : 0;
    __syncthreads();
    sh[threadIdx.x] += add;
    __syncthreads();
  }
  if (i < len) a[i] = sh[threadIdx.x] - v;
  if (threadIdx.x == 1023) bsum[blockIdx.x] = sh[1023];
}

__global__ __launch_bounds__(1024) void scan_sums_kernel(int32_t* __restrict__ bsum, int nb) {
  __shared__ int32_t sh[1024];
  int32_t carry = 0;
  for (int base = 0; base < nb; base += 1024) {
    const int i = base + threadIdx.x;
    const int32_t v = i < nb ? bsum[i] : 0;
    sh[threadIdx.x] = v;
    __syncthreads();
    for (int off = 1; off < 1024; off <<= 1) {
      const int32_t add = threadIdx.x >= off ? sh[threadIdx.x - off] : 0;
      __syncthreads();
      sh[threadIdx.x] += add;
      __syncthreads();
    }
    if (i < nb) bsum[i] = carry + sh[threadIdx.x] - v;
    const int32_t tot = sh[1023];
    __syncthreads();
    carry += tot;
  }
}

__global__ __launch_bounds__(1024) void scan_add_kernel(int32_t* __restrict__ a, int64_t len,
                                                        const int32_t* __restrict__ bsum) {
  const int64_t i = (int64_t)blockIdx.x * 1024 + threadIdx.x;
  if (i < len) a[i] += bsum[blockIdx.x];
}

__global__ void grid_scatter_kernel(int64_t n, const double* __restrict__ sx,
                                    const double* __restrict__ sy,
                                    const int32_t* __restrict__ key,
                                    const int32_t* __restrict__ off, int32_t* __restrict__ fill,
                                    double* __restrict__ px, double* __restrict__ py,
                                    int32_t* __restrict__ pidx) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  const int k = key[i];
  const int pos = off[k] + atomicAdd(&fill[k], 1);
  if (px) {
    px[pos] = sx[i];
    py[pos] = sy[i];
  }
  pidx[pos] = (int32_t)i;
}

// The scatter leaves each cell's points in arrival order; sorting every cell by
// point index makes the processing order built from the grid independent of
// scheduling (the neighbor search itself does not depend on the order inside a
// cell). One wavefront per cell: the cell's indices are staged in LDS and each
// is written back at its rank (the count of smaller indices in the cell);
// cells longer than kCellCap take a heapsort by one lane instead.
constexpr int kCellCap = 1024;

__global__ __launch_bounds__(256) void cell_sort_kernel(int64_t ncells,
                                                        const int32_t* __restrict__ off,
                                                        int32_t* __restrict__ pidx) {
  __shared__ int32_t sbuf[4][kCellCap];
  const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
  const int64_t c = (int64_t)blockIdx.x * 4 + wave;
  if (c >= ncells) return;  // whole wavefront; no workgroup barriers below
  int32_t* a = pidx + off[c];
  const int len = off[c + 1] - off[c];
  if (len < 2) return;
  if (len <= kCellCap) {
    int32_t* buf = sbuf[wave];
    for (int q = lane; q < len; q += 64) buf[q] = a[q];
    wave_lds_sync();
    for (int q = lane; q < len; q += 64) {
      const int32_t v = buf[q];
      int rank = 0;
      for (int r = 0; r < len; ++r) rank += buf[r] < v ? 1 : 0;
      a[rank] = v;
    }
    return;
  }
  if (lane != 0) return;
  auto sift = [&](int root, int end) {
    while (2 * root + 1 < end) {
      int child = 2 * root + 1;
      if (child + 1 < end && a[child] < a[child + 1]) ++child;
      if (a[root] >= a[child]) return;
      const int32_t tmp = a[root];
      a[root] = a[child];
      a[child] = tmp;
      root = child;
    }
  };
  for (int st = len / 2 - 1; st >= 0; --st) sift(st, len);
  for (int end = len - 1; end > 0; --end) {
    const int32_t tmp = a[0];
    a[0] = a[end];
    a[end] = tmp;
    sift(0, end);
  }
}


// Ranking keys. Fixed operation order and no contraction, so that any IEEE FP64
// implementation of the same sequence returns the same bits.
template <int MODE>
__device__ __forceinline__ double rank_key(double dx, double dy, double t1, double t2,
                                           const NbrArgs& A) {
#pragma clang fp contract(off)
  if (MODE == 1) {
    double u = dx * A.ir_s;
    double v = dy * A.ir_s;
    double s = u * u + v * v;
    return -(t1 + s);
  }
  double h2 = dx * dx + dy * dy;
  if (MODE == 0) {
    double g = sqrt(h2);
    return -(t1 + g * t2);
  }
  if (MODE == 2) {
    double g = pow(h2, A.gamma);
    return -(t1 + g * t2);
  }
  double x = sqrt(h2) * t2;
  double s = A.nu_code == 1 ? x - log1p(x) : x - log1p(x + x * x / 3.0);
  s = s > 0.0 ? s : 0.0;
  return -(t1 + s);
}

// Lag-only factors of the key at the real lag l >= 0 (general times), in the
// operation order of the per-lag tables the host computes for integer times.
__device__ __forceinline__ void lag_factors(const NbrArgs& A, double l, double& f1, double& f2) {
#pragma clang fp contract(off)
  if (A.mode == 1) {
    const double w = l * A.ir_t;
    f1 = w * w;
    f2 = 0.0;
    return;
  }
  const double psi = A.a * pow(l, A.two_alpha) + 1.0;
  f1 = A.c1 * log(psi);
  f2 = A.c * pow(psi, A.e2);
}

// Upper bound of the key over candidates at distance >= d (d already reduced by
// the slack): the same operation sequence as rank_key at that distance.
template <int MODE>
__device__ __forceinline__ double bound_key(double d, double t1, double t2, const NbrArgs& A) {
#pragma clang fp contract(off)
  if (MODE == 1) {
    double u = d * A.ir_s;
    return -(t1 + u * u);
  }
  if (MODE == 0) return -(t1 + d * t2);
  if (MODE == 2) return -(t1 + pow(d * d, A.gamma) * t2);
  double x = d * t2;
  double s = A.nu_code == 1 ? x - log1p(x) : x - log1p(x + x * x / 3.0);
  s = s > 0.0 ? s : 0.0;
  return -(t1 + s);
}

// Rank order of candidates: larger key first, then lower index.
__device__ __forceinline__ bool ranks_before(double ka, int ia, double kb, int ib) {
  return ka > kb || (ka == kb && ia < ib);
}

// Compare-exchange with lane ^ stride; the lower lane keeps the better pair
// when `desc`, the worse one otherwise.
__device__ __forceinline__ void cmpx(double& k, int& id, int lane, int stride, bool desc) {
  const double pk = __shfl_xor(k, stride);
  const int pi = __shfl_xor(id, stride);
  const bool lower = (lane & stride) == 0;
  const bool pb = ranks_before(pk, pi, k, id);
  const bool take = (lower == desc) ? pb : !pb;
  k = take ? pk : k;
  id = take ? pi : id;
}

// Bitonic sort of one (key, index) pair per lane into rank order (lane 0 best).
__device__ __forceinline__ void wave_sort64(double& k, int& id, int lane) {
#pragma unroll
  for (int size = 2; size <= 64; size <<= 1)
#pragma unroll
    for (int stride = size >> 1; stride > 0; stride >>= 1)
      cmpx(k, id, lane, stride, (lane & size) == 0 || size == 64);
}

// Rank-order a bitonic sequence held one pair per lane.
__device__ __forceinline__ void wave_merge64(double& k, int& id, int lane) {
#pragma unroll
  for (int stride = 32; stride > 0; stride >>= 1) cmpx(k, id, lane, stride, true);
}

// Offer one chunk of candidates (one per lane) to the running top-m list.
__device__ __forceinline__ void offer(double key, int j, bool valid, double& K, int& I, int& cnt,
                                      double& thr, int& thr_i, int lane, int m) {
  const bool better = valid && (cnt < m || key > thr || (key == thr && j < thr_i));
  unsigned long long mask = __ballot(better);
  const int nsurv = __popcll(mask);
  if (nsurv > 8) {
    // Many survivors: sort them across the wave and merge with the list. The
    // list and the reversed sorted chunk form a bitonic sequence whose
    // lane-wise better halves are the best 64 of the union.
    double ck = better ? key : -INFINITY;
    int cj = better ? j : INT_MAX;
    wave_sort64(ck, cj, lane);
    const double rk = __shfl(ck, 63 - lane);
    const int rj = __shfl(cj, 63 - lane);
    if (ranks_before(rk, rj, K, I)) {
      K = rk;
      I = rj;
    }
    wave_merge64(K, I, lane);
    cnt = cnt + nsurv < m ? cnt + nsurv : m;
    if (cnt >= m) {
      thr = __shfl(K, m - 1);
      thr_i = __shfl(I, m - 1);
    }
    return;
  }
  while (mask) {
    const int s = __ffsll((long long)mask) - 1;
    mask &= mask - 1;
    const double ck = __shfl(key, s);
    const int cj = __shfl(j, s);
    if (cnt >= m && !(ck > thr || (ck == thr && cj < thr_i))) continue;
    const bool before = lane < cnt && (K > ck || (K == ck && I < cj));
    const int pos = __popcll(__ballot(before));
    const double pK = __shfl_up(K, 1);
    const int pI = __shfl_up(I, 1);
    if (lane == pos) {
      K = ck;
      I = cj;
    } else if (lane > pos) {
      K = pK;
      I = pI;
    }
    if (cnt < m) ++cnt;
    if (cnt >= m) {
      thr = __shfl(K, m - 1);
      thr_i = __shfl(I, m - 1);
    }
  }
}

// Key and offer the candidates of ring r around cell (qcx, qcy) of one slab: the
// top and bottom rows of the ring as one CSR range each, the rows between as
// their two end cells. The ranges (wave-uniform bounds) fill 64-lane chunks one
// after another, a chunk spanning several ranges, and the last chunk of the ring
// is offered partly filled, so the ring's candidates take as few offers as their
// count allows.
template <int MODE, bool GENERAL>
__device__ __forceinline__ void scan_ring(const NbrArgs& A, const GridArgs& G, const int32_t* off,
                                          int qcx, int qcy, int r, double qx, double qy, double qt,
                                          double t1, double t2, int jmax, double& K, int& I,
                                          int& cnt, double& thr, int& thr_i, int lane, int m) {
  int p = -1;      // this lane's candidate position in the CSR arrays, -1 if none
  int filled = 0;  // lanes of the current chunk already assigned
  auto flush = [&]() {
    const bool inrun = p >= 0;
    const int j = inrun ? G.pidx[p] : INT_MAX;
    const bool valid = inrun && j < jmax;
    double key = -INFINITY;
    if (valid) {
      if constexpr (GENERAL) {
        double f1, f2;
        lag_factors(A, qt - A.t[j], f1, f2);
        key = rank_key<MODE>(G.px[p] - qx, G.py[p] - qy, f1, f2, A);
      } else {
        key = rank_key<MODE>(G.px[p] - qx, G.py[p] - qy, t1, t2, A);
      }
    }
    offer(key, j, valid, K, I, cnt, thr, thr_i, lane, m);
    p = -1;
    filled = 0;
  };
  auto add = [&](int beg, int end) {
    while (beg < end) {
      const int take = end - beg < 64 - filled ? end - beg : 64 - filled;
      if (lane >= filled && lane < filled + take) p = beg + (lane - filled);
      filled += take;
      beg += take;
      if (filled == 64) flush();
    }
  };
  const int y0 = qcy - r, y1 = qcy + r;
  const int ya = y0 < 0 ? 0 : y0, yb = y1 >= G.gy ? G.gy - 1 : y1;
  const int xa = qcx - r < 0 ? 0 : qcx - r, xb = qcx + r >= G.gx ? G.gx - 1 : qcx + r;
  for (int cy = ya; cy <= yb; ++cy) {
    const int32_t* o = off + cy * G.gx;
    if (cy == y0 || cy == y1) {
      add(o[xa], o[xb + 1]);  // top or bottom row of the ring: one contiguous run
    } else {
      if (qcx - r >= 0) add(o[qcx - r], o[qcx - r + 1]);
      if (qcx + r < G.gx) add(o[qcx + r], o[qcx + r + 1]);
    }
  }
  if (filled > 0) flush();
}

// One wavefront per query; the register budget is held to seven waves per SIMD
// (measured faster than six, and eight spills).
// GENERAL (real-valued times): a slab is a time bin; the tables hold, per bin lag
// L, the lag factors at the smallest and largest lag two bins L apart can have
// (f1 nondecreasing, f2 nonincreasing in the lag), so both bounds hold for every
// pair of those bins; since each pair's own factors come from the device math
// library, the comparisons with the bounds keep a relative slack of 1e-12.
template <int MODE, bool GENERAL>
__global__ __launch_bounds__(256, 7) void neighbors_grid_kernel(NbrArgs A, GridArgs G) {
  const int lane = threadIdx.x & 63;
  const int64_t w = (int64_t)blockIdx.x * 4 + (threadIdx.x >> 6);
  if (w >= A.n) return;  // uniform per wave
  const int64_t i = A.qlist ? (int64_t)A.qlist[w] : w;
  const int m = A.m;
  const double qx = A.sx[i], qy = A.sy[i], qt = A.t[i];
  const int ti = GENERAL ? min((int)((qt - A.t0) * A.islab), G.nslab - 1) : (int)(qt - A.t0);
  auto slack = [](double b) { return GENERAL ? b + 1e-12 * (1.0 + fabs(b)) : b; };
  const int qcx = cell_of(qx, G.xmin, G.icw, G.gx);
  const int qcy = cell_of(qy, G.ymin, G.ich, G.gy);
  double K = -INFINITY;
  int I = INT_MAX;
  int cnt = 0;
  double thr = -INFINITY;
  int thr_i = INT_MAX;
  for (int lag = 0; lag <= ti; ++lag) {
    if (cnt >= m && slack(A.bnd[lag]) < thr) break;
    const int slab = ti - lag;
    const int32_t* off = G.off + (int64_t)slab * G.ncell;
    const int jmax = (lag == 0) ? (int)i : INT_MAX;
    const double t1 = A.tab1[lag], t2 = A.tab2[lag];
    for (int r = 0;; ++r) {
      if (r > 0) {
        // Everything not yet visited lies outside the block of cells within
        // Chebyshev distance r - 1; d is the distance to that block's edges.
        const int bx0 = qcx - (r - 1), bx1 = qcx + (r - 1);
        const int by0 = qcy - (r - 1), by1 = qcy + (r - 1);
        double d = INFINITY;
        if (bx0 > 0) d = fmin(d, qx - (G.xmin + bx0 * G.cw));
        if (bx1 < G.gx - 1) d = fmin(d, (G.xmin + (bx1 + 1) * G.cw) - qx);
        if (by0 > 0) d = fmin(d, qy - (G.ymin + by0 * G.ch));
        if (by1 < G.gy - 1) d = fmin(d, (G.ymin + (by1 + 1) * G.ch) - qy);
        if (d == INFINITY) break;  // the grid is covered
        if (cnt >= m) {
          const double ds = fmax(0.0, d * (1.0 - 1e-9) - G.margin);
          if (slack(bound_key<MODE>(ds, t1, t2, A)) < thr) break;
        }
      }
      scan_ring<MODE, GENERAL>(A, G, off, qcx, qcy, r, qx, qy, qt, t1, t2, jmax, K, I, cnt, thr,
                               thr_i, lane, m);
    }
  }
  if (lane < m) A.nbr[i * m + lane] = lane < cnt ? I : -1;
}

}  // namespace

hipError_t launch_validate_times(int64_t n, const double* t, uint32_t* flag, hipStream_t s) {
  if (n <= 0) return hipSuccess;
  unsigned grid = (unsigned)((n + 255) / 256);
  hipLaunchKernelGGL(validate_times_kernel, dim3(grid), dim3(256), 0, s, n, t, flag);
  return hipGetLastError();
}

hipError_t launch_bbox(int64_t n, const double* sx, const double* sy, double* partial,
                       double* out, hipStream_t s) {
  hipLaunchKernelGGL(bbox_stage1, dim3(kRedBlocks), dim3(256), 0, s, n, sx, sy, partial);
  hipLaunchKernelGGL(bbox_stage2, dim3(1), dim3(256), 0, s, (const double*)partial, out);
  return hipGetLastError();
}

hipError_t launch_exclusive_scan(int32_t* a, int64_t len, int32_t* bsum, hipStream_t s) {
  if (len <= 0) return hipSuccess;
  const int nb = (int)((len + 1023) / 1024);
  hipLaunchKernelGGL(scan_tiles_kernel, dim3(nb), dim3(1024), 0, s, a, len, bsum);
  hipLaunchKernelGGL(scan_sums_kernel, dim3(1), dim3(1024), 0, s, bsum, nb);
  hipLaunchKernelGGL(scan_add_kernel, dim3(nb), dim3(1024), 0, s, a, len, (const int32_t*)bsum);
  return hipGetLastError();
}

hipError_t launch_grid_build(int64_t n, const double* sx, const double* sy, const double* t,
                             double t0, const GridArgs& g, int32_t* counts, int32_t* fill,
                             int32_t* bsum, int32_t* key, double* px, double* py, int32_t* pidx,
                             hipStream_t s) {
  const int64_t len = (int64_t)g.nslab * g.ncell + 1;
  const unsigned gl = (unsigned)((len + 255) / 256);
  const unsigned gn = (unsigned)((n + 255) / 256);
  hipLaunchKernelGGL(fill_i32_kernel, dim3(gl), dim3(256), 0, s, counts, len);
  hipLaunchKernelGGL(fill_i32_kernel, dim3(gl), dim3(256), 0, s, fill, len);
  hipLaunchKernelGGL(grid_count_kernel, dim3(gn), dim3(256), 0, s, n, sx, sy, t, t0, g, counts,
                     key);
  const int nb = (int)((len + 1023) / 1024);
  hipLaunchKernelGGL(scan_tiles_kernel, dim3(nb), dim3(1024), 0, s, counts, len, bsum);
  hipLaunchKernelGGL(scan_sums_kernel, dim3(1), dim3(1024), 0, s, bsum, nb);
  hipLaunchKernelGGL(scan_add_kernel, dim3(nb), dim3(1024), 0, s, counts, len,
                     (const int32_t*)bsum);
  hipLaunchKernelGGL(grid_scatter_kernel, dim3(gn), dim3(256), 0, s, n, sx, sy,
                     (const int32_t*)key, (const int32_t*)counts, fill, px, py, pidx);
  if (!px) {
    // processing order: made independent of scheduling
    const int64_t ncells = len - 1;
    hipLaunchKernelGGL(cell_sort_kernel, dim3((unsigned)((ncells + 3) / 4)), dim3(256), 0, s,
                       ncells, (const int32_t*)counts, pidx);
  }
  return hipGetLastError();
}

// ------------------------------------------------------- candidate proposal ----
// One wavefront per query. The window (earlier points of slabs t_i - lags .. t_i
// in the grid cells within r of the query's in x and y, r the smallest radius in
// 1..rmax whose cells hold at least wmin points of those slabs, counted from the
// cell offsets with the query's whole slab, else rmax) is scored -- squared embedding
// distance in FP32 (dimension order, no contraction) or squared spatial distance
// in FP64 -- into LDS; a bitonic sort on (score, index) picks the ncand best;
// their exact ranking keys (the key of the exact search) are sorted on
// (key descending, index ascending) and the first m written. Windows smaller
// than min(i, m) or larger than cmax set the row's fallback flag instead.
__device__ __forceinline__ float emb_dist(const float* __restrict__ ei,
                                          const float* __restrict__ ej) {
#pragma clang fp contract(off)
  float acc = 0.f;
#pragma unroll
  for (int k = 0; k < 16; ++k) {
    const float d = ei[k] - ej[k];
    const float d2 = d * d;
    acc = acc + d2;
  }
  return acc;
}

__device__ __forceinline__ double spatial_dist(double dx, double dy) {
#pragma clang fp contract(off)
  const double a = dx * dx;
  const double b = dy * dy;
  return a + b;
}

// (ka, ia) before (kb, ib) in ascending score order, ties to the lower index.
__device__ __forceinline__ bool asc_before(uint64_t ka, int ia, uint64_t kb, int ib) {
  return ka < kb || (ka == kb && ia < ib);
}

template <int MODE>
__global__ __launch_bounds__(256) void propose_kernel(NbrArgs A, GridArgs G, ProposeArgs P) {
  constexpr int CM = kProposeCmax;
  __shared__ uint64_t sk[4][CM];
  __shared__ int32_t si[4][CM];
  const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
  const int64_t i = (int64_t)blockIdx.x * 4 + wv;
  if (i >= A.n) return;  // uniform per wave
  uint64_t* K = sk[wv];
  int32_t* I = si[wv];
  const int m = A.m;
  const double qx = A.sx[i], qy = A.sy[i];
  const int ti = (int)(A.t[i] - A.t0);
  const int qcx = cell_of(qx, G.xmin, G.icw, G.gx);
  const int qcy = cell_of(qy, G.ymin, G.ich, G.gy);
  float ei[16];
  if (P.E) {
#pragma unroll
    for (int k = 0; k < 16; ++k) ei[k] = P.E[i * 16 + k];
  }
  int cnt = 0;
  const int lmax = P.lags < ti ? P.lags : ti;
  // points of the slabs in the cells within radius r (CSR offsets; rows of cells
  // are contiguous), summed over the wave
  auto count_r = [&](int r) {
    const int ny = 2 * r + 1;
    const int cx0 = qcx - r < 0 ? 0 : qcx - r;
    const int cx1 = qcx + r >= G.gx ? G.gx - 1 : qcx + r;
    int part = 0;
    for (int e = lane; e < ny * (lmax + 1); e += 64) {
      const int lag = e / ny, cy = qcy - r + (e - lag * ny);
      if (cy < 0 || cy >= G.gy) continue;
      const int32_t* off = G.off + (int64_t)(ti - lag) * G.ncell + (int64_t)cy * G.gx;
      part += off[cx1 + 1] - off[cx0];
    }
#pragma unroll
    for (int sh = 32; sh > 0; sh >>= 1) part += __shfl_xor(part, sh);
    return part;
  };
  int rad = P.rmax;
  if (count_r(1) >= P.wmin) {
    rad = 1;
  } else {
    int lo = 1, hi = P.rmax;  // count(lo) < wmin; find the smallest r with count >= wmin
    if (count_r(hi) >= P.wmin) {
      while (hi - lo > 1) {
        const int mid = (lo + hi) >> 1;
        if (count_r(mid) >= P.wmin) hi = mid; else lo = mid;
      }
    }
    rad = hi;
  }
  for (int lag = 0; lag <= lmax; ++lag) {
    const int slab = ti - lag;
    const int32_t* off = G.off + (int64_t)slab * G.ncell;
    for (int cy = qcy - rad; cy <= qcy + rad; ++cy) {
      if (cy < 0 || cy >= G.gy) continue;
      const int cx0 = qcx - rad < 0 ? 0 : qcx - rad;
      const int cx1 = qcx + rad >= G.gx ? G.gx - 1 : qcx + rad;
      // cells cx0..cx1 of one row are contiguous in the CSR order
      const int beg = off[cy * G.gx + cx0], end = off[cy * G.gx + cx1 + 1];
      for (int b0 = beg; b0 < end; b0 += 64) {
        const int pos = b0 + lane;
        bool ok = pos < end;
        int j = 0;
        uint64_t key = 0;
        if (ok) {
          j = G.pidx[pos];
          ok = lag > 0 || (int64_t)j < i;
        }
        if (ok) {
          if (P.E) {
            const float d = emb_dist(ei, P.Ecsr + (int64_t)pos * 16);
            key = (uint64_t)__float_as_uint(d);
          } else {
            key = (uint64_t)__double_as_longlong(spatial_dist(G.px[pos] - qx, G.py[pos] - qy));
          }
        }
        const unsigned long long bal = __ballot(ok);
        const int at = cnt + __popcll(bal & ((1ull << lane) - 1ull));
        if (ok && at < CM) {
          K[at] = key;
          I[at] = j;
        }
        cnt += __popcll(bal);
      }
    }
  }
  const int need = (int64_t)m < i ? m : (int)i;
  if (cnt < need || cnt > P.cmax) {
    if (lane == 0) P.fallback[i] = 1;
    return;
  }
  if (lane == 0) P.fallback[i] = 0;
  // pad to a power of two and sort ascending on (score, index)
  int L2 = 1;
  while (L2 < cnt) L2 <<= 1;
  for (int e = cnt + lane; e < L2; e += 64) {
    K[e] = ~0ull;
    I[e] = INT_MAX;
  }
  wave_lds_sync();
  for (int kk = 2; kk <= L2; kk <<= 1) {
    for (int jj = kk >> 1; jj > 0; jj >>= 1) {
      for (int e = lane; e < L2; e += 64) {
        const int pt = e ^ jj;
        if (pt > e) {
          const uint64_t ka = K[e], kb = K[pt];
          const int ia = I[e], ib = I[pt];
          const bool up = (e & kk) == 0;
          if (asc_before(kb, ib, ka, ia) == up) {
            K[e] = kb; I[e] = ib;
            K[pt] = ka; I[pt] = ia;
          }
        }
      }
      wave_lds_sync();
    }
  }
  // exact keys of the first nc candidates, two per lane
  const int nc = cnt < P.ncand ? cnt : P.ncand;
  double kx[2];
  int jx[2];
#pragma unroll
  for (int h = 0; h < 2; ++h) {
    const int e = lane + 64 * h;
    kx[h] = -INFINITY;
    jx[h] = INT_MAX;
    if (e < nc) {
      const int j = I[e];
      const int lj = ti - (int)(A.t[j] - A.t0);
      kx[h] = rank_key<MODE>(A.sx[j] - qx, A.sy[j] - qy, A.tab1[lj], A.tab2[lj], A);
      jx[h] = j;
    }
  }
  wave_lds_sync();
  // sort the 128 (key, index) pairs on (key descending, index ascending) in LDS
  double* DK = reinterpret_cast<double*>(K);
#pragma unroll
  for (int h = 0; h < 2; ++h) {
    DK[lane + 64 * h] = kx[h];
    I[lane + 64 * h] = jx[h];
  }
  wave_lds_sync();
  for (int kk = 2; kk <= 128; kk <<= 1) {
    for (int jj = kk >> 1; jj > 0; jj >>= 1) {
#pragma unroll
      for (int h = 0; h < 2; ++h) {
        const int e = lane + 64 * h;
        const int pt = e ^ jj;
        if (pt > e) {
          const double ka = DK[e], kb = DK[pt];
          const int ia = I[e], ib = I[pt];
          const bool up = (e & kk) == 0;
          if (ranks_before(kb, ib, ka, ia) == up) {
            DK[e] = kb; I[e] = ib;
            DK[pt] = ka; I[pt] = ia;
          }
        }
      }
      wave_lds_sync();
    }
  }
  if (lane < m) A.nbr[i * m + lane] = lane < nc ? I[lane] : -1;
}

__global__ void permute16_kernel(int64_t n, const int32_t* __restrict__ pidx,
                                 const float* __restrict__ E, float* __restrict__ out) {
  const int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (e >= n * 4) return;
  const int64_t pos = e >> 2;
  const int q = (int)(e & 3);
  reinterpret_cast<float4*>(out)[pos * 4 + q] =
      reinterpret_cast<const float4*>(E)[(int64_t)pidx[pos] * 4 + q];
}

__global__ void compact_kernel(int64_t n, const int32_t* __restrict__ flag,
                               int32_t* __restrict__ list, int32_t* __restrict__ count) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n || !flag[i]) return;
  list[atomicAdd(count, 1)] = (int32_t)i;
}

hipError_t launch_neighbors(const NbrArgs& a, const GridArgs& g, hipStream_t s) {
  if (a.n <= 0 || a.m <= 0) return hipSuccess;
  unsigned grid = (unsigned)((a.n + 3) / 4);
  if (a.general) {
    switch (a.mode) {
      case 0: hipLaunchKernelGGL((neighbors_grid_kernel<0, true>), dim3(grid), dim3(256), 0, s, a, g); break;
      case 1: hipLaunchKernelGGL((neighbors_grid_kernel<1, true>), dim3(grid), dim3(256), 0, s, a, g); break;
      case 2: hipLaunchKernelGGL((neighbors_grid_kernel<2, true>), dim3(grid), dim3(256), 0, s, a, g); break;
      default: hipLaunchKernelGGL((neighbors_grid_kernel<3, true>), dim3(grid), dim3(256), 0, s, a, g); break;
    }
    return hipGetLastError();
  }
  switch (a.mode) {
    case 0: hipLaunchKernelGGL((neighbors_grid_kernel<0, false>), dim3(grid), dim3(256), 0, s, a, g); break;
    case 1: hipLaunchKernelGGL((neighbors_grid_kernel<1, false>), dim3(grid), dim3(256), 0, s, a, g); break;
    case 2: hipLaunchKernelGGL((neighbors_grid_kernel<2, false>), dim3(grid), dim3(256), 0, s, a, g); break;
    default: hipLaunchKernelGGL((neighbors_grid_kernel<3, false>), dim3(grid), dim3(256), 0, s, a, g); break;
  }
  return hipGetLastError();
}

hipError_t launch_propose(const NbrArgs& a, const GridArgs& g, const ProposeArgs& pa,
                          hipStream_t s) {
  if (a.n <= 0 || a.m <= 0) return hipSuccess;
  const unsigned grid = (unsigned)((a.n + 3) / 4);
  switch (a.mode) {
    case 0: hipLaunchKernelGGL(propose_kernel<0>, dim3(grid), dim3(256), 0, s, a, g, pa); break;
    case 1: hipLaunchKernelGGL(propose_kernel<1>, dim3(grid), dim3(256), 0, s, a, g, pa); break;
    case 2: hipLaunchKernelGGL(propose_kernel<2>, dim3(grid), dim3(256), 0, s, a, g, pa); break;
    default: hipLaunchKernelGGL(propose_kernel<3>, dim3(grid), dim3(256), 0, s, a, g, pa); break;
  }
  return hipGetLastError();
}

hipError_t launch_compact(int64_t n, const int32_t* flag, int32_t* list, int32_t* count,
                          hipStream_t s) {
  if (n <= 0) return hipSuccess;
  hipLaunchKernelGGL(compact_kernel, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, s, n, flag,
                     list, count);
  return hipGetLastError();
}

hipError_t launch_zero_i32(int32_t* p, int64_t cnt, hipStream_t s) {
  if (cnt <= 0) return hipSuccess;
  hipLaunchKernelGGL(fill_i32_kernel, dim3((unsigned)((cnt + 255) / 256)), dim3(256), 0, s, p, cnt);
  return hipGetLastError();
}

hipError_t launch_permute16(int64_t n, const int32_t* pidx, const float* E, float* out,
                            hipStream_t s) {
  if (n <= 0) return hipSuccess;
  hipLaunchKernelGGL(permute16_kernel, dim3((unsigned)((n * 4 + 255) / 256)), dim3(256), 0, s, n,
                     pidx, E, out);
  return hipGetLastError();
}

}  // namespace vif
