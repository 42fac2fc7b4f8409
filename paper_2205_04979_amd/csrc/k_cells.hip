// Cell-list neighbour search and short-range pair forces: soft-sphere normal
// contact (Appendix A.2.2) and van der Waals cohesion (Eq. vdw, Appendix A.2.3).
//
// Build (after the histogram made by k_prepare): exclusive scan of the cell
// counts -> scatter with per-cell atomic slots -> per-cell ascending sort of
// the particle indices, so the neighbour walk and hence every force sum runs
// in a fixed order (bitwise reproducible).  The sort pass also clears the
// counts for the next build, so no memset is ever enqueued.
#include "common.hpp"
#include "launch.hpp"

namespace depo {

constexpr int SCAN_THREADS = 256;
constexpr int SCAN_PER_THREAD = 4;
constexpr int SCAN_BLOCK = SCAN_THREADS * SCAN_PER_THREAD;

__device__ __forceinline__ int block_exclusive_scan(int v, int *sh, int &total) {
  const int t = threadIdx.x;
  sh[t] = v;
  __syncthreads();
  for (int off = 1; off < SCAN_THREADS; off <<= 1) {
    int add = t >= off ? sh[t - off] : 0;
    __syncthreads();
    sh[t] += add;
    __syncthreads();
  }
  total = sh[SCAN_THREADS - 1];
  int excl = sh[t] - v;
  __syncthreads();
  return excl;
}

__global__ __launch_bounds__(SCAN_THREADS) void k_scan_reduce(const int32_t *__restrict__ count, int n,
                                                              int32_t *__restrict__ part) {
  __shared__ int sh[SCAN_THREADS];
  const int base = blockIdx.x * SCAN_BLOCK + threadIdx.x * SCAN_PER_THREAD;
  int v = 0;
#pragma unroll
  for (int k = 0; k < SCAN_PER_THREAD; ++k) v += base + k < n ? count[base + k] : 0;
  int total;
  block_exclusive_scan(v, sh, total);
  if (threadIdx.x == 0) part[blockIdx.x] = total;
}

__global__ __launch_bounds__(SCAN_THREADS) void k_scan_top(int32_t *__restrict__ part, int nb,
                                                           int32_t *__restrict__ start, int n) {
  __shared__ int sh[SCAN_THREADS];
  int carry = 0;
  for (int b0 = 0; b0 < nb; b0 += SCAN_THREADS) {
    const int b = b0 + threadIdx.x;
    const int v = b < nb ? part[b] : 0;
    int total;
    const int ex = block_exclusive_scan(v, sh, total);
    if (b < nb) part[b] = carry + ex;
    carry += total;
  }
  if (threadIdx.x == 0) start[n] = carry;
}

__global__ __launch_bounds__(SCAN_THREADS) void k_scan_apply(int32_t *__restrict__ count, int n,
                                                             const int32_t *__restrict__ part,
                                                             int32_t *__restrict__ start) {
  __shared__ int sh[SCAN_THREADS];
  const int base = blockIdx.x * SCAN_BLOCK + threadIdx.x * SCAN_PER_THREAD;
  int c[SCAN_PER_THREAD];
  int v = 0;
#pragma unroll
  for (int k = 0; k < SCAN_PER_THREAD; ++k) {
    c[k] = base + k < n ? count[base + k] : 0;
    v += c[k];
  }
  int total;
  int run = block_exclusive_scan(v, sh, total) + part[blockIdx.x];
#pragma unroll
  for (int k = 0; k < SCAN_PER_THREAD; ++k)
    if (base + k < n) {
      start[base + k] = run;
      count[base + k] = 0;
      run += c[k];
    }
}

__global__ __launch_bounds__(256) void k_scatter(const int32_t *__restrict__ cell_of, int N,
                                                 const int32_t *__restrict__ start, int32_t *__restrict__ count,
                                                 int32_t *__restrict__ idx) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= N) return;
  const int c = cell_of[i];
  if (c < 0) return;
  const int slot = start[c] + atomicAdd(&count[c], 1);
  idx[slot] = i;
}

__global__ __launch_bounds__(256) void k_cell_sort(const int32_t *__restrict__ start, int n_cells,
                                                   int32_t *__restrict__ count, int32_t *__restrict__ idx) {
  const int c = blockIdx.x * blockDim.x + threadIdx.x;
  if (c >= n_cells) return;
  const int b = start[c], e = start[c + 1];
  for (int k = b + 1; k < e; ++k) {
    const int v = idx[k];
    int j = k - 1;
    while (j >= b && idx[j] > v) {
      idx[j + 1] = idx[j];
      --j;
    }
    idx[j + 1] = v;
  }
  count[c] = 0;
}

__global__ void k_clear_int(int32_t *p, size_t n) {
  const size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) p[i] = 0;
}

// Cohesive force magnitude of two spheres (diameters di, dj) at surface gap
// gs: -dU/dr of Hamaker's two-sphere energy, written as the single product
// (32/3) A R1^3 R2^3 r / (P^2 Q^2), P = r^2 - (R1+R2)^2 = gs (gs + 2 (R1+R2)),
// Q = r^2 - (R1-R2)^2, which equals Eq. vdw for equal spheres.  Lengths are
// handled in micrometres so that every intermediate stays in FP32 range.
template <class Real>
__device__ __forceinline__ Real vdw_force(Real gs_m, Real di_m, Real dj_m, Real A) {
  const Real u = Real(1e6);
  const Real r1 = Real(0.5) * di_m * u, r2 = Real(0.5) * dj_m * u, g = gs_m * u;
  const Real s = r1 + r2, t = r1 - r2;
  const Real r = s + g;
  const Real P = g * (g + Real(2) * s);
  const Real Q = (r - t) * (r + t);
  const Real r13 = r1 * r1 * r1, r23 = r2 * r2 * r2;
  const Real PQ = P * Q;
  return Real(32.0 / 3.0) * A * u * (r13 * r23) * r / (PQ * PQ);
}

// One thread per alive particle, taken in cell order (the sorted index array),
// so the threads of a wavefront walk neighbouring cells and share their loads.
// Removed particles are not visited; their short-range slots are never read.
template <class Real>
__global__ __launch_bounds__(256) void k_short_range(State<Real> st, Phys ph, int n_cells) {
  const int t = blockIdx.x * blockDim.x + threadIdx.x;
  if (t >= st.cell_start[n_cells]) return;
  const int i = st.cell_idx[t];
  const SampleDev sp = st.samples[st.sid[i]];
  const auto px = st.px[i], py = st.py[i], pz = st.pz[i];
  const double rxi = st.rx[i], ryi = st.ry[i], rzi = st.rz[i];
  const Real vix = st.vx[i], viy = st.vy[i], viz = st.vz[i];
  int cx, cy, cz, mx, my, mz;
  short_range_cells(px, py, pz, sp, cx, cy, cz, mx, my, mz);
  const double di_d = st.d[i];
  const Real di = Real(di_d);
  const Real mi = Real(ph.mass_coef) * di * di * di;
  const Real A = Real(sp.hamaker);
  const Real dsat = Real(ph.delta_sat);
  const bool vdw = (ph.flags & F_VDW) != 0, col = (ph.flags & F_COLLIDE) != 0;
  Real a0 = 0, a1 = 0, a2 = 0;
  int nb = 0;
  // only the neighbour cells whose shared face is closer than the reach can hold a partner
  for (int ox = -1; ox <= 1; ++ox) {
    if ((ox < 0 && !(mx & 1)) || (ox > 0 && !(mx & 2))) continue;
    int xx = cx + ox;
    xx = xx < 0 ? xx + sp.ncx : (xx >= sp.ncx ? xx - sp.ncx : xx);
    for (int oy = -1; oy <= 1; ++oy) {
      if ((oy < 0 && !(my & 1)) || (oy > 0 && !(my & 2))) continue;
      const int yy = cy + oy;
      if (yy < 0 || yy >= sp.ncy) continue;
      for (int oz = -1; oz <= 1; ++oz) {
        if ((oz < 0 && !(mz & 1)) || (oz > 0 && !(mz & 2))) continue;
        const int zz = cz + oz;
        if (zz < 0 || zz >= sp.ncz) continue;
        const int c = sp.cell_base + (xx * sp.ncy + yy) * sp.ncz + zz;
        const int e = st.cell_start[c + 1];
        for (int k = st.cell_start[c]; k < e; ++k) {
          const int j = st.cell_idx[k];
          if (j == i) continue;
          // geometry and the range test in FP64 (the gap near contact is a small fraction of |r|)
          const double dj_d = st.d[j];
          double gx, gy, gz, gd;
          const double gap_d = pair_gap(px, py, pz, st.px[j], st.py[j], st.pz[j], rxi - (double)st.rx[j],
                                        ryi - (double)st.ry[j], rzi - (double)st.rz[j], ph.ux, ph.ur,
                                        0.5 * (di_d + dj_d), gx, gy, gz, gd);
          if (gap_d > 0.25 * fmin(di_d, dj_d) || gd == 0.0) continue;
          ++nb;
          const double inv_d = 1.0 / gd;
          const Real nx = Real(gx * inv_d), ny = Real(gy * inv_d), nz = Real(gz * inv_d);
          const Real dj = Real(dj_d);
          const Real gap = Real(gap_d);
          Real f = 0;   // along +n (away from j), per unit mass of i
          if (vdw) f -= vdw_force(fmax(gap, dsat), di, dj, A) / mi;
          if (col && gap < Real(0)) {
            const Real mj = Real(ph.mass_coef) * dj * dj * dj;
            const Real vn = (vix - st.vx[j]) * nx + (viy - st.vy[j]) * ny + (viz - st.vz[j]) * nz;
            f += mj / (mi + mj) * (Real(ph.col_K) * (-gap) - Real(ph.col_H) * vn);
          }
          a0 += f * nx; a1 += f * ny; a2 += f * nz;
        }
      }
    }
  }
  st.sx[i] = a0; st.sy[i] = a1; st.sz[i] = a2;
  st.nbr[i] = nb;
}

template <class Real>
void launch_cells(const State<Real> &st, const Phys &ph, int n_cells, int n_scan_blocks, hipStream_t s) {
  hipLaunchKernelGGL(k_scan_reduce, dim3(n_scan_blocks), dim3(SCAN_THREADS), 0, s, st.cell_count, n_cells,
                     st.scan_part);
  hipLaunchKernelGGL(k_scan_top, dim3(1), dim3(SCAN_THREADS), 0, s, st.scan_part, n_scan_blocks, st.cell_start,
                     n_cells);
  hipLaunchKernelGGL(k_scan_apply, dim3(n_scan_blocks), dim3(SCAN_THREADS), 0, s, st.cell_count, n_cells,
                     st.scan_part, st.cell_start);
  if (ph.N > 0)
    hipLaunchKernelGGL(k_scatter, dim3((ph.N + 255) / 256), dim3(256), 0, s, st.cell_of, ph.N, st.cell_start,
                       st.cell_count, st.cell_idx);
  hipLaunchKernelGGL(k_cell_sort, dim3((n_cells + 255) / 256), dim3(256), 0, s, st.cell_start, n_cells,
                     st.cell_count, st.cell_idx);
}

template <class Real>
void launch_short_range(const State<Real> &st, const Phys &ph, int n_cells, hipStream_t s) {
  if (ph.N > 0) hipLaunchKernelGGL(k_short_range<Real>, dim3((ph.N + 255) / 256), dim3(256), 0, s, st, ph, n_cells);
}

void launch_clear_int(int32_t *p, size_t n, hipStream_t s) {
  if (n) hipLaunchKernelGGL(k_clear_int, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, s, p, n);
}

template void launch_cells<float>(const State<float> &, const Phys &, int, int, hipStream_t);
template void launch_cells<double>(const State<double> &, const Phys &, int, int, hipStream_t);
template void launch_short_range<float>(const State<float> &, const Phys &, int, hipStream_t);
template void launch_short_range<double>(const State<double> &, const Phys &, int, hipStream_t);

}  // namespace depo
