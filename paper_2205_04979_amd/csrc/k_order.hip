// Storage order of the particles.  When enabled, the per-particle state is
// permuted into the order of the last cell list at the start of every step
// that follows a multiple of `every` steps: particles of one cell, and of
// neighbouring cells, then sit in neighbouring slots, so the cell-ordered walks
// (short-range pairs, cell build) and the field gather read contiguous rows
// instead of one cache line per particle and field.  Every sample keeps its
// slot range: its alive particles first, in cell order (within a cell by slot,
// as the cell list sorts them), then its removed particles in slot order.  The
// permutation is deterministic.  perm[] travels with the particles, so the
// host returns everything in the caller's order.
//
// The kernels are part of every captured step and decide on the device, from
// the step counter, whether this step reorders (otherwise they return at once).
// Passes: the inverse of the cell list (into cell_of, free at a step's start),
// a count and scan of removed particles per block of slots, the scatter into
// the scratch copy, and the copy back (the captured step keeps fixed array
// addresses).
#include "common.hpp"
#include "launch.hpp"

namespace depo {

namespace {

constexpr int kThreads = 256;
constexpr int kPer = 4;                       // slots per thread, kThreads apart (consecutive lanes, consecutive slots)
constexpr int kBlock = kThreads * kPer;       // slots per block of the count and scatter passes

__device__ __forceinline__ bool due(const int32_t *nstep, int every) {
  const int n = *nstep;
  return every > 0 && n > 0 && n % every == 0;
}

// exclusive scan of one value per thread over a block of kThreads threads
__device__ __forceinline__ int block_scan(int v, int *sh, int &total) {
  const int t = threadIdx.x;
  sh[t] = v;
  __syncthreads();
  for (int off = 1; off < kThreads; off <<= 1) {
    const int add = t >= off ? sh[t - off] : 0;
    __syncthreads();
    sh[t] += add;
    __syncthreads();
  }
  total = sh[kThreads - 1];
  const int ex = sh[t] - v;
  __syncthreads();
  return ex;
}

// pos[i] = position of alive particle i in the cell list
template <class Real>
__global__ __launch_bounds__(kThreads) void k_order_inverse(State<Real> st, int n_cells, int every) {
  if (!due(st.nstep, every)) return;
  const int k = blockIdx.x * blockDim.x + threadIdx.x;
  if (k >= st.cell_start[n_cells]) return;
  st.cell_of[st.cell_idx[k]] = k;
}

// removed particles per block of kBlock slots
template <class Real>
__global__ __launch_bounds__(kThreads) void k_order_count(State<Real> st, int n, int every) {
  if (!due(st.nstep, every)) return;
  __shared__ int sh[kThreads];
  const int base = blockIdx.x * kBlock + threadIdx.x;
  int c = 0;
#pragma unroll
  for (int q = 0; q < kPer; ++q) {
    const int i = base + q * kThreads;
    c += (i < n && st.dep[i] != 0) ? 1 : 0;
  }
  int total;
  block_scan(c, sh, total);
  if (threadIdx.x == 0) st.scan_part[blockIdx.x] = total;
}

// exclusive scan of the block counts (one workgroup)
template <class Real>
__global__ __launch_bounds__(kThreads) void k_order_top(State<Real> st, int nb, int every) {
  if (!due(st.nstep, every)) return;
  __shared__ int sh[kThreads];
  int carry = 0;
  for (int b0 = 0; b0 < nb; b0 += kThreads) {
    const int b = b0 + threadIdx.x;
    const int v = b < nb ? st.scan_part[b] : 0;
    int total;
    const int ex = block_scan(v, sh, total);
    if (b < nb) st.scan_part[b] = carry + ex;
    carry += total;
  }
}

// new slot of every particle, and its state into the scratch copy there
template <class Real>
__global__ __launch_bounds__(kThreads) void k_order_scatter(State<Real> st, OrderScratch<Real> sc, int n, int every) {
  if (!due(st.nstep, every)) return;
  __shared__ int sh[kThreads];
  const int base = blockIdx.x * kBlock + threadIdx.x;
  int run = st.scan_part[blockIdx.x];   // removed particles in the slots before this row of the block
#pragma unroll
  for (int q = 0; q < kPer; ++q) {
    const int i = base + q * kThreads;
    const bool dead = i < n && st.dep[i] != 0;
    int total;
    const int rank = run + block_scan(dead ? 1 : 0, sh, total);   // removed particles in slots < i
    run += total;
    if (i >= n) continue;
    const SampleDev sp = st.samples[st.sid[i]];
    const int a0 = st.cell_start[sp.cell_base];                              // alive before the sample
    const int a1 = st.cell_start[sp.cell_base + sp.ncx * sp.ncy * sp.ncz];   // ... and up to its end
    int k;
    if (dead) {
      // alive slots of the sample first, then its removed particles in slot order; sp.start - a0
      // removed particles precede the sample
      k = sp.start + (a1 - a0) + (rank - (sp.start - a0));
    } else {
      k = sp.start + (st.cell_of[i] - a0);
    }
    if (k < sp.start || k >= sp.start + sp.count) {   // a cell list that does not describe the storage
      atomicOr(st.err, ERR_ORDER);
      continue;
    }
    sc.px[k] = st.px[i]; sc.py[k] = st.py[i]; sc.pz[k] = st.pz[i];
    sc.rx[k] = st.rx[i]; sc.ry[k] = st.ry[i]; sc.rz[k] = st.rz[i];
    sc.vx[k] = st.vx[i]; sc.vy[k] = st.vy[i]; sc.vz[k] = st.vz[i];
    sc.ax[k] = st.ax[i]; sc.ay[k] = st.ay[i]; sc.az[k] = st.az[i];
    sc.ux[k] = st.ux[i]; sc.uy[k] = st.uy[i]; sc.uz[k] = st.uz[i];
    sc.jr[k] = st.jr[i];
    sc.d[k] = st.d[i]; sc.qb[k] = st.qb[i]; sc.ell[k] = st.ell[i];
    sc.dep[k] = st.dep[i]; sc.nbr[k] = st.nbr[i]; sc.perm[k] = st.perm[i];
  }
}

template <class Real>
__global__ __launch_bounds__(kThreads) void k_order_copy(State<Real> st, OrderScratch<Real> sc, int n, int every) {
  if (!due(st.nstep, every)) return;
  const int k = blockIdx.x * blockDim.x + threadIdx.x;
  if (k >= n) return;
  st.px[k] = sc.px[k]; st.py[k] = sc.py[k]; st.pz[k] = sc.pz[k];
  st.rx[k] = sc.rx[k]; st.ry[k] = sc.ry[k]; st.rz[k] = sc.rz[k];
  st.vx[k] = sc.vx[k]; st.vy[k] = sc.vy[k]; st.vz[k] = sc.vz[k];
  st.ax[k] = sc.ax[k]; st.ay[k] = sc.ay[k]; st.az[k] = sc.az[k];
  st.ux[k] = sc.ux[k]; st.uy[k] = sc.uy[k]; st.uz[k] = sc.uz[k];
  st.jr[k] = sc.jr[k];
  st.d[k] = sc.d[k]; st.qb[k] = sc.qb[k]; st.ell[k] = sc.ell[k];
  st.dep[k] = sc.dep[k]; st.nbr[k] = sc.nbr[k]; st.perm[k] = sc.perm[k];
}

}  // namespace

template <class Real>
void launch_order(const State<Real> &st, const OrderScratch<Real> &sc, int n, int n_cells, int every, hipStream_t s) {
  if (n <= 0 || every <= 0) return;
  const unsigned g = (unsigned)((n + kThreads - 1) / kThreads);
  const int nb = (n + kBlock - 1) / kBlock;
  hipLaunchKernelGGL((k_order_inverse<Real>), dim3(g), dim3(kThreads), 0, s, st, n_cells, every);
  hipLaunchKernelGGL((k_order_count<Real>), dim3((unsigned)nb), dim3(kThreads), 0, s, st, n, every);
  hipLaunchKernelGGL((k_order_top<Real>), dim3(1), dim3(kThreads), 0, s, st, nb, every);
  hipLaunchKernelGGL((k_order_scatter<Real>), dim3((unsigned)nb), dim3(kThreads), 0, s, st, sc, n, every);
  hipLaunchKernelGGL((k_order_copy<Real>), dim3(g), dim3(kThreads), 0, s, st, sc, n, every);
}

template void launch_order<float>(const State<float> &, const OrderScratch<float> &, int, int, int, hipStream_t);
template void launch_order<double>(const State<double> &, const OrderScratch<double> &, int, int, int, hipStream_t);

}  // namespace depo
