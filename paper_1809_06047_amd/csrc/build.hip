// Generic build step on gfx950: from a mesh matrix M to its edge ids and
// adjacency, i.e. the mapped products E = M M^T {Q_c + Q_c^{c-1}} (eq:CC_E)
// and F = M M^T {Q_c}[gamma] (eq:F), computed without forming the product
// (Sec. 4.2): every collision of M(i,k) with M^T(k,j) is a pair of cyclic
// neighbours i, j inside face k, so the work is organised per vertex over
// the faces it touches.
//
//   1. valence n = M 1 (eq:vo) by integer atomics, plus input validation
//   2. exclusive scan of n -> row pointer of the row view of M
//   3. incidence fill: the half-edges leaving each vertex (a transpose of M
//      by atomic cursors; rows are sorted afterwards so nothing depends on
//      atomic order)
//   4. per vertex: twin half-edges (the F pattern), boundary starts, fan
//      check, and the sorted set of lower neighbours (the column of the
//      strict upper triangle of E owned by this vertex); its size is the
//      symbolic count of Sec. 4.2
//   5. exclusive scan of the counts -> column pointer of triu(E) = edge base
//   6. per vertex: edge id = base[hi] + rank of lo (CSC enumeration of the
//      upper triangle), edge -> half-edge map, boundary flags (E == 1)
// plus the crease matrix C placed onto edge ids (Sec. 3.3) and the device
// exclusive scan used by every step.
#include <climits>

#include "subdiv_internal.h"

namespace subdiv {

// ------------------------------------------------------------------ fills
__global__ void k_fill_i32(int32_t *p, int32_t value, long long n) {
  long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  const long long stride = (long long)gridDim.x * blockDim.x;
  for (; i < n; i += stride) p[i] = value;
}

hipError_t launch_fill_i32(int32_t *p, int32_t value, long long n, hipStream_t s) {
  if (n <= 0) return hipSuccess;
  unsigned g = grid_for(n);
  if (g > 8192) g = 8192;
  hipLaunchKernelGGL(k_fill_i32, dim3(g), dim3(kBlock), 0, s, p, value, n);
  return hipGetLastError();
}

// several regions cleared to zero by one launch (the build's counters and
// crease tables: each launch of its own would add its own latency)
__global__ void k_zero_regions(ZeroRegions z) {
  const long long stride = (long long)gridDim.x * blockDim.x;
  for (int r = 0; r < z.count; ++r)
    for (long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x; i < z.n[r]; i += stride) z.p[r][i] = 0;
}

hipError_t launch_zero_regions(const ZeroRegions &z, hipStream_t s) {
  long long m = 0;
  for (int r = 0; r < z.count; ++r) m = z.n[r] > m ? z.n[r] : m;
  if (m <= 0) return hipSuccess;
  unsigned g = grid_for(m);
  if (g > 8192) g = 8192;
  hipLaunchKernelGGL(k_zero_regions, dim3(g), dim3(kBlock), 0, s, z);
  return hipGetLastError();
}

hipError_t launch_fill_u8(uint8_t *p, long long nbytes, hipStream_t s) {
  // callers only clear 4-byte aligned regions whose size is a multiple of 4
  return launch_fill_i32(reinterpret_cast<int32_t *>(p), 0, nbytes / 4, s);
}

// Vertex data of `dim` channels, row-major [V*dim]: three channels at a time
// go through the position kernels as a [V*3] array. pack: channels c0..c0+2
// (those past dim read as zero).
__global__ void k_pack3(const float *data, int dim, int c0, long long n3, float *slice) {
  const long long x = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  if (x >= n3) return;
  const long long v = x / 3;
  const int c = c0 + (int)(x - 3 * v);
  slice[x] = c < dim ? data[v * dim + c] : 0.0f;
}

hipError_t launch_pack3(const float *data, int dim, int c0, long long V, float *slice, hipStream_t s) {
  if (V <= 0) return hipSuccess;
  hipLaunchKernelGGL(k_pack3, dim3(grid_for(3 * V)), dim3(kBlock), 0, s, data, dim, c0, 3 * V, slice);
  return hipGetLastError();
}

// channels c0 .. c0+ncols-1 (ncols <= 6) of out from two [V*3] arrays
// holding channels c0..c0+2 and c0+3..c0+5: one lane per output value, so
// when the group spans every channel each row is written whole, by
// consecutive lanes
// The group width is a template argument and the index 32-bit when it fits,
// so the row/column split is a multiply by a constant, not a 64-bit divide.
template <int NC, typename I>
__global__ void k_unpack6(const float *__restrict__ a, const float *__restrict__ b, int dim, int c0, I n,
                          float *__restrict__ out) {
  const I x = (I)blockIdx.x * blockDim.x + threadIdx.x;
  if (x >= n) return;
  const I v = x / NC;
  const int c = (int)(x - v * NC);
  const float y = c < 3 ? a[3 * v + c] : b[3 * v + c - 3];
  __builtin_nontemporal_store(y, out + (long long)v * dim + c0 + c);
}

template <int NC>
static void unpack_t(const float *a, const float *b, int dim, int c0, long long V, float *out, hipStream_t s) {
  const long long n = V * NC;
  if (n <= 0xffffffffll)
    hipLaunchKernelGGL((k_unpack6<NC, uint32_t>), dim3(grid_for(n)), dim3(kBlock), 0, s, a, b, dim, c0, (uint32_t)n,
                       out);
  else
    hipLaunchKernelGGL((k_unpack6<NC, long long>), dim3(grid_for(n)), dim3(kBlock), 0, s, a, b, dim, c0, n, out);
}

hipError_t launch_unpack6(const float *a, const float *b, int dim, int c0, int ncols, long long V, float *out,
                          hipStream_t s) {
  if (V <= 0) return hipSuccess;
  switch (ncols) {
    case 1: unpack_t<1>(a, b, dim, c0, V, out, s); break;
    case 2: unpack_t<2>(a, b, dim, c0, V, out, s); break;
    case 3: unpack_t<3>(a, b, dim, c0, V, out, s); break;
    case 4: unpack_t<4>(a, b, dim, c0, V, out, s); break;
    case 5: unpack_t<5>(a, b, dim, c0, V, out, s); break;
    case 6: unpack_t<6>(a, b, dim, c0, V, out, s); break;
    default: return hipErrorInvalidValue;
  }
  return hipGetLastError();
}

// ------------------------------------------------------------------- scan
// Block-wide scans: 256 threads x 8 items. A wave-64 inclusive scan with
// cross-lane shuffles, then the 4 wave totals through LDS. Inputs of at most
// kScanSmall items are scanned by one 1024-thread block in a single launch
// (a few tiles with a running carry): the plan of a cage and the small levels
// are bound by launch latency, not by the scan's bytes.
constexpr int kScanThreads = 256;
constexpr int kScanItems = 8;
constexpr int kScanTile = kScanThreads * kScanItems;
constexpr int kScanOneThreads = 1024;
constexpr int kScanOneTile = kScanOneThreads * 16;
constexpr long long kScanSmall = 2ll * kScanOneTile;

__device__ __forceinline__ int wave_incl_scan(int v) {
  const int lane = threadIdx.x & 63;
#pragma unroll
  for (int d = 1; d < 64; d <<= 1) {
    const int y = __shfl_up(v, d, 64);
    if (lane >= d) v += y;
  }
  return v;
}

// Exclusive scan of one value per thread across a block of NT threads;
// *total = block sum.
template <int NT = kScanThreads>
__device__ __forceinline__ int block_excl_scan(int x, int *total) {
  __shared__ int wsum[NT / 64];
  const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6;
  const int incl = wave_incl_scan(x);
  if (lane == 63) wsum[wid] = incl;
  __syncthreads();
  int off = 0, tot = 0;
#pragma unroll
  for (int w = 0; w < NT / 64; ++w) {
    const int s = wsum[w];
    off += (w < wid) ? s : 0;
    tot += s;
  }
  __syncthreads();
  *total = tot;
  return off + incl - x;
}

// A thread's 8 consecutive items as two 16-byte loads when they are all in
// range and the array is 16-byte aligned (VEC), else one by one.
template <bool VEC>
__device__ __forceinline__ void load8(const int32_t *in, long long base, long long n, int (&v)[kScanItems]) {
  if (VEC && base + kScanItems <= n) {
    const int4 a = reinterpret_cast<const int4 *>(in + base)[0], b = reinterpret_cast<const int4 *>(in + base)[1];
    v[0] = a.x; v[1] = a.y; v[2] = a.z; v[3] = a.w;
    v[4] = b.x; v[5] = b.y; v[6] = b.z; v[7] = b.w;
  } else {
#pragma unroll
    for (int i = 0; i < kScanItems; ++i) v[i] = (base + i < n) ? in[base + i] : 0;
  }
}

template <bool VEC>
__global__ void __launch_bounds__(kScanThreads) k_scan_reduce(const int32_t *in, long long n, int32_t *partials) {
  const long long base = (long long)blockIdx.x * kScanTile + (long long)threadIdx.x * kScanItems;
  int v[kScanItems];
  load8<VEC>(in, base, n, v);
  int s = 0;
#pragma unroll
  for (int i = 0; i < kScanItems; ++i) s += v[i];
  int tot;
  block_excl_scan(s, &tot);
  if (threadIdx.x == 0) partials[blockIdx.x] = tot;
}

// single block: exclusive scan of partials[0..nb) in place, partials[nb] = total
__global__ void __launch_bounds__(kScanThreads) k_scan_partials(int32_t *partials, long long nb) {
  int carry = 0;
  for (long long t0 = 0; t0 < nb; t0 += kScanTile) {
    const long long base = t0 + (long long)threadIdx.x * kScanItems;
    int v[kScanItems];
    int s = 0;
#pragma unroll
    for (int i = 0; i < kScanItems; ++i) {
      v[i] = (base + i < nb) ? partials[base + i] : 0;
      s += v[i];
    }
    int tot;
    int off = block_excl_scan(s, &tot) + carry;
#pragma unroll
    for (int i = 0; i < kScanItems; ++i) {
      if (base + i < nb) partials[base + i] = off;
      off += v[i];
    }
    carry += tot;
  }
  if (threadIdx.x == 0) partials[nb] = carry;
}

template <bool VEC>
__global__ void __launch_bounds__(kScanThreads) k_scan_apply(const int32_t *in, int32_t *out, long long n,
                                                            const int32_t *partials, long long nb,
                                                            int32_t *total_dst) {
  const long long base = (long long)blockIdx.x * kScanTile + (long long)threadIdx.x * kScanItems;
  int v[kScanItems];
  load8<VEC>(in, base, n, v);
  int s = 0;
#pragma unroll
  for (int i = 0; i < kScanItems; ++i) s += v[i];
  int tot;
  int off = block_excl_scan(s, &tot) + (partials ? partials[blockIdx.x] : 0);
  if (VEC && base + kScanItems <= n) {
    int o[kScanItems];
#pragma unroll
    for (int i = 0; i < kScanItems; ++i) {
      o[i] = off;
      off += v[i];
    }
    reinterpret_cast<int4 *>(out + base)[0] = make_int4(o[0], o[1], o[2], o[3]);
    reinterpret_cast<int4 *>(out + base)[1] = make_int4(o[4], o[5], o[6], o[7]);
  } else {
#pragma unroll
    for (int i = 0; i < kScanItems; ++i) {
      if (base + i < n) out[base + i] = off;
      off += v[i];
    }
  }
  if (blockIdx.x == gridDim.x - 1 && threadIdx.x == kScanThreads - 1) {
    const int total = partials ? partials[nb] : off;
    out[n] = total;
    if (total_dst) *total_dst = total;
  }
}

// one block: the whole scan of n <= kScanSmall items (in may equal out: every
// tile is read into registers before it is written)
__global__ void __launch_bounds__(kScanOneThreads) k_scan_one(const int32_t *in, int32_t *out, long long n,
                                                              int32_t *total_dst) {
  constexpr int kI = kScanOneTile / kScanOneThreads;
  static_assert(kI % 4 == 0, "a thread's items are whole int4s");
  // a thread's items as int4 loads and stores when both arrays are 16-byte
  // aligned and its items are all in range (one by one they leave every lane
  // of an instruction on a different line)
  const bool vec = reinterpret_cast<uintptr_t>(in) % 16 == 0 && reinterpret_cast<uintptr_t>(out) % 16 == 0;
  int carry = 0;
  for (long long t0 = 0; t0 < n; t0 += kScanOneTile) {
    const long long base = t0 + (long long)threadIdx.x * kI;
    const bool whole = vec && base + kI <= n;
    int v[kI];
    int s = 0;
    if (whole) {
#pragma unroll
      for (int q = 0; q < kI / 4; ++q) {
        const int4 x = reinterpret_cast<const int4 *>(in + base)[q];
        v[4 * q] = x.x;
        v[4 * q + 1] = x.y;
        v[4 * q + 2] = x.z;
        v[4 * q + 3] = x.w;
      }
    } else {
#pragma unroll
      for (int i = 0; i < kI; ++i) v[i] = (base + i < n) ? in[base + i] : 0;
    }
#pragma unroll
    for (int i = 0; i < kI; ++i) s += v[i];
    int tot;
    int off = block_excl_scan<kScanOneThreads>(s, &tot) + carry;
    int o[kI];
#pragma unroll
    for (int i = 0; i < kI; ++i) {
      o[i] = off;
      off += v[i];
    }
    if (whole) {
#pragma unroll
      for (int q = 0; q < kI / 4; ++q)
        reinterpret_cast<int4 *>(out + base)[q] = make_int4(o[4 * q], o[4 * q + 1], o[4 * q + 2], o[4 * q + 3]);
    } else {
#pragma unroll
      for (int i = 0; i < kI; ++i)
        if (base + i < n) out[base + i] = o[i];
    }
    carry += tot;
  }
  if (threadIdx.x == 0) {
    out[n] = carry;
    if (total_dst) *total_dst = carry;
  }
}

long long scan_partials_ints(long long n) { return (n + kScanTile - 1) / kScanTile + 1; }

hipError_t launch_scan(const int32_t *in, int32_t *out, long long n, int32_t *partials, int32_t *total_dst,
                       hipStream_t s) {
  const long long nb = (n + kScanTile - 1) / kScanTile;
  if (nb <= 1) {
    hipLaunchKernelGGL(k_scan_apply<false>, dim3(1), dim3(kScanThreads), 0, s, in, out, n, (const int32_t *)nullptr,
                       0ll, total_dst);
    return hipGetLastError();
  }
  if (n <= kScanSmall) {
    hipLaunchKernelGGL(k_scan_one, dim3(1), dim3(kScanOneThreads), 0, s, in, out, n, total_dst);
    return hipGetLastError();
  }
  const bool vec = reinterpret_cast<uintptr_t>(in) % 16 == 0 && reinterpret_cast<uintptr_t>(out) % 16 == 0;
  if (vec) {
    hipLaunchKernelGGL(k_scan_reduce<true>, dim3((unsigned)nb), dim3(kScanThreads), 0, s, in, n, partials);
  } else {
    hipLaunchKernelGGL(k_scan_reduce<false>, dim3((unsigned)nb), dim3(kScanThreads), 0, s, in, n, partials);
  }
  hipLaunchKernelGGL(k_scan_partials, dim3(1), dim3(kScanThreads), 0, s, partials, nb);
  if (vec) {
    hipLaunchKernelGGL(k_scan_apply<true>, dim3((unsigned)nb), dim3(kScanThreads), 0, s, in, out, n,
                       (const int32_t *)partials, nb, total_dst);
  } else {
    hipLaunchKernelGGL(k_scan_apply<false>, dim3((unsigned)nb), dim3(kScanThreads), 0, s, in, out, n,
                       (const int32_t *)partials, nb, total_dst);
  }
  return hipGetLastError();
}

// ------------------------------------------------------------------ build
// 1. per face: validation, valence atomics, column of every non-zero
template <int ORDER>
__global__ void k_build_faces(Topo t, int scheme, int32_t *nval, int32_t *hface_out, DeviceInfo *info) {
  const int f = blockIdx.x * blockDim.x + threadIdx.x;
  if (f >= t.F) return;
  uint32_t fault = 0;
  int b, e;
  if constexpr (ORDER > 0) {
    b = f * ORDER;
    e = b + ORDER;
  } else {
    b = t.off[f];
    e = t.off[f + 1];
    if (f == 0 && b != 0) fault |= FAULT_INVALID_ARG;
    if (f == t.F - 1 && e != t.H) fault |= FAULT_INVALID_ARG;
    if (e < b || b < 0 || e > t.H) {
      atomicOr(&info->faults, fault | FAULT_INVALID_ARG);
      return;
    }
  }
  const int c = e - b;
  if (c < 3) fault |= FAULT_DEGENERATE;
  if (scheme != SUBDIV_CATMULL_CLARK && c != 3) fault |= FAULT_SCHEME_MESH;
  for (int h = b; h < e; ++h) {
    const int v = t.fv[h];
    if (hface_out) hface_out[h] = f;
    if (v < 0 || v >= t.V) {
      fault |= FAULT_INVALID_ARG;
      continue;
    }
    atomicAdd(&nval[v], 1);
    for (int g = b; g < h; ++g)
      if (t.fv[g] == v) fault |= FAULT_DEGENERATE;
  }
  if (fault) atomicOr(&info->faults, fault);
}

// The kernels after the validation pass run in the same stream without a
// host round trip; once any fault is recorded they do nothing (indices of an
// invalid cage may be out of range), and the plan reports the fault. The
// faults that matter were recorded by earlier kernels of the stream, whose
// writes every later kernel sees, so a plain (cached, uniform) load is
// enough; a volatile one sent every lane's load to memory and made a large
// cage's build twice as slow.
__device__ __forceinline__ bool faulted(const DeviceInfo *info) { return info->faults != 0; }

// 3. row view of M: half-edges leaving each vertex
__global__ void k_build_incidence(Topo t, const int32_t *rowptr, int32_t *cursor, int32_t *inc,
                                  const DeviceInfo *info) {
  const int h = blockIdx.x * blockDim.x + threadIdx.x;
  if (h >= t.H || faulted(info)) return;
  const int v = t.fv[h];
  const int pos = atomicAdd(&cursor[v], 1);
  inc[rowptr[v] + pos] = h;
}

// in-place insertion sort of a short int list (per-thread, global memory)
__device__ void sort_small(int32_t *a, int n) {
  for (int i = 1; i < n; ++i) {
    const int x = a[i];
    int j = i - 1;
    while (j >= 0 && a[j] > x) {
      a[j + 1] = a[j];
      --j;
    }
    a[j + 1] = x;
  }
}

// Batcher's odd-even merge sort of N (a power of two) values held in
// registers: the loops unroll into a fixed network of min/max pairs.
template <int N>
__device__ __forceinline__ void sort_net(int (&a)[N]) {
#pragma unroll
  for (int p = 1; p < N; p <<= 1)
#pragma unroll
    for (int k = p; k >= 1; k >>= 1)
#pragma unroll
      for (int j = k % p; j + k < N; j += 2 * k)
#pragma unroll
        for (int i = 0; i < k; ++i)
          if (i + j + k < N && (i + j) / (2 * p) == (i + j + k) / (2 * p)) {
            const int x = a[i + j], y = a[i + j + k];
            a[i + j] = min(x, y);
            a[i + j + k] = max(x, y);
          }
}

constexpr int kRegValence = 8;  // rows up to this valence are handled in registers

// 4. per vertex: twins, boundary start, fan check, lower neighbours.
// Register path for valence <= kRegValence: the row and the end points of
// its half-edges are loaded once, side by side, and every search runs on
// registers.
template <int ORDER>
__device__ void vertex_row_regs(const Topo &t, int v, int r0, int n, int32_t *inc, int32_t *cand, int32_t *twin,
                                int32_t *vhe, int32_t *cntlo, DeviceInfo *info) {
  constexpr int R = kRegValence;
  int hh[R];
#pragma unroll
  for (int i = 0; i < R; ++i) hh[i] = i < n ? inc[r0 + i] : INT_MAX;
  sort_net<R>(hh);
  int pv[R], ww[R], uu[R];
#pragma unroll
  for (int i = 0; i < R; ++i) {
    const bool ok = i < n;
    const int nx = ok ? he_next<ORDER>(t, hh[i]) : 0;
    pv[i] = ok ? he_prev<ORDER>(t, hh[i]) : 0;
    ww[i] = ok ? t.fv[nx] : -1;     // h = v -> w
    uu[i] = ok ? t.fv[pv[i]] : -2;  // prev(h) = u -> v
  }
  uint32_t fault = 0;
  int start = hh[0], start_u = uu[0], nbnd = 0;
#pragma unroll
  for (int i = 0; i < R; ++i) {
    if (i < n) {
      int tw = -1, hits = 0;
#pragma unroll
      for (int m = 0; m < R; ++m)
        if (uu[m] == ww[i]) {  // prev(row[m]) runs w -> v: the twin of v -> w
          tw = pv[m];
          ++hits;
        }
      if (hits > 1) fault |= FAULT_NONMANIFOLD;
#pragma unroll
      for (int m = 0; m < i; ++m)
        if (ww[m] == ww[i]) fault |= FAULT_NONMANIFOLD;  // directed edge v->w twice
      twin[hh[i]] = tw;
      if (tw < 0) {
        if (nbnd == 0) {
          start = hh[i];
          start_u = uu[i];
        }
        ++nbnd;
      }
      inc[r0 + i] = hh[i];  // the sorted row
    }
  }
  if (nbnd > 1) fault |= FAULT_NONMANIFOLD;
  vhe[v] = start;
  // one fan: from the start, the next half-edge leaves v towards u = prev's source
  int steps = 0, cu = start_u;
  for (int it = 0; it < R + 1; ++it) {
    ++steps;
    if (steps > n) break;
    int hn = -1, nu = 0;
#pragma unroll
    for (int m = 0; m < R; ++m)
      if (ww[m] == cu) {
        hn = hh[m];
        nu = uu[m];
      }
    if (hn < 0 || hn == start) break;
    cu = nu;
  }
  if (steps != n) fault |= FAULT_NONMANIFOLD;
  // lower neighbours (one column of triu(E)), sorted and distinct
  int c[2 * R];
#pragma unroll
  for (int i = 0; i < R; ++i) {
    c[2 * i] = (i < n && ww[i] < v) ? ww[i] : INT_MAX;
    c[2 * i + 1] = (i < n && uu[i] >= 0 && uu[i] < v) ? uu[i] : INT_MAX;
  }
  sort_net<2 * R>(c);
  int32_t *out = cand + 2 * r0;
  int d = 0;
#pragma unroll
  for (int i = 0; i < 2 * R; ++i)
    if (c[i] != INT_MAX && (i == 0 || c[i] != c[i - 1])) out[d++] = c[i];
  cntlo[v] = d;
  if (fault) atomicOr(&info->faults, fault);
}

// General path (any valence): the same steps on the row in global memory.
template <int ORDER>
__device__ void vertex_row_general(const Topo &t, int v, int r0, int n, int32_t *inc, int32_t *cand, int32_t *twin,
                                   int32_t *vhe, int32_t *cntlo, DeviceInfo *info) {
  uint32_t fault = 0;
  int32_t *row = inc + r0;
  sort_small(row, n);
  int start = row[0], nbnd = 0;
  for (int i = 0; i < n; ++i) {
    const int h = row[i];
    const int w = t.fv[he_next<ORDER>(t, h)];
    int tw = -1, hits = 0;
    for (int m = 0; m < n; ++m) {
      const int hp = he_prev<ORDER>(t, row[m]);
      if (t.fv[hp] == w) {
        tw = hp;
        ++hits;
      }
    }
    if (hits > 1) fault |= FAULT_NONMANIFOLD;
    for (int m = 0; m < i; ++m)
      if (t.fv[he_next<ORDER>(t, row[m])] == w) fault |= FAULT_NONMANIFOLD;  // directed edge v->w twice
    twin[h] = tw;
    if (tw < 0) {
      if (nbnd == 0) start = h;
      ++nbnd;
    }
  }
  if (nbnd > 1) fault |= FAULT_NONMANIFOLD;
  vhe[v] = start;
  // one fan: walk from the start around v through twin(prev(h))
  int steps = 0, h = start;
  while (true) {
    ++steps;
    if (steps > n) break;
    const int u = t.fv[he_prev<ORDER>(t, h)];
    int hn = -1;
    for (int m = 0; m < n; ++m)
      if (t.fv[he_next<ORDER>(t, row[m])] == u) hn = row[m];
    if (hn < 0 || hn == start) break;
    h = hn;
  }
  if (steps != n) fault |= FAULT_NONMANIFOLD;
  // lower neighbours (one column of triu(E)), sorted and distinct
  int32_t *c = cand + 2 * r0;
  int k = 0;
  for (int i = 0; i < n; ++i) {
    const int w = t.fv[he_next<ORDER>(t, row[i])];
    const int u = t.fv[he_prev<ORDER>(t, row[i])];
    if (w < v) c[k++] = w;
    if (u < v) c[k++] = u;
  }
  sort_small(c, k);
  int d = 0;
  for (int i = 0; i < k; ++i)
    if (i == 0 || c[i] != c[i - 1]) c[d++] = c[i];
  cntlo[v] = d;
  if (fault) atomicOr(&info->faults, fault);
}

template <int ORDER>
__global__ void k_build_vertex(Topo t, const int32_t *rowptr, int32_t *inc, int32_t *cand, int32_t *twin,
                               int32_t *vhe, int32_t *cntlo, DeviceInfo *info) {
  const int v = blockIdx.x * blockDim.x + threadIdx.x;
  const bool live = v < t.V && !faulted(info);
  const int r0 = live ? rowptr[v] : 0, n = live ? rowptr[v + 1] - r0 : 0;
  // the largest valence: reduced over the wave first, one atomic per wave
  // (one per vertex on a single word serialises a large cage's build)
  int vmax = n;
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) vmax = max(vmax, __shfl_xor(vmax, o, 64));
  if ((threadIdx.x & 63) == 0 && vmax > 0) atomicMax(&info->max_valence, vmax);
  if (!live) return;
  if (n == 0 || n > SUBDIV_MAX_VALENCE) {
    atomicOr(&info->faults, n == 0 ? FAULT_DEGENERATE : FAULT_INVALID_ARG);
    vhe[v] = -1;
    cntlo[v] = 0;
    return;
  }
  if (n <= kRegValence) vertex_row_regs<ORDER>(t, v, r0, n, inc, cand, twin, vhe, cntlo, info);
  else vertex_row_general<ORDER>(t, v, r0, n, inc, cand, twin, vhe, cntlo, info);
}

__device__ __forceinline__ int rank_of(const int32_t *c, int n, int x) {
  int lo = 0, hi = n;
  while (lo < hi) {
    const int m = (lo + hi) >> 1;
    if (c[m] < x) lo = m + 1;
    else hi = m;
  }
  return lo;
}

// 6. edge ids (CSC order of triu(E)), edge -> half-edge, boundary flags
template <int ORDER>
__global__ void k_build_eid(Topo t, const int32_t *rowptr, const int32_t *inc, const int32_t *cand,
                            const int32_t *cntlo, const int32_t *ebase, const int32_t *twin, int32_t *eid,
                            int32_t *e2h, int32_t *bflag, DeviceInfo *info) {
  const int v = blockIdx.x * blockDim.x + threadIdx.x;
  if (v >= t.V || faulted(info)) return;
  const int r0 = rowptr[v], n = rowptr[v + 1] - r0;
  const int32_t *c = cand + 2 * r0;
  const int cnt = cntlo[v], base = ebase[v];
  int nb = 0;
  if (n <= kRegValence) {
    // register path: the row, its end points, twins and the lower neighbours
    // are loaded side by side; ranks are counted on registers
    constexpr int R = kRegValence;
    int hh[R], pv[R], ww[R], uu[R], cc[2 * R];
#pragma unroll
    for (int i = 0; i < R; ++i) {
      const bool ok = i < n;
      hh[i] = ok ? inc[r0 + i] : 0;
      pv[i] = ok ? he_prev<ORDER>(t, hh[i]) : 0;
      ww[i] = ok ? t.fv[he_next<ORDER>(t, hh[i])] : INT_MAX;
      uu[i] = ok ? t.fv[pv[i]] : INT_MAX;
    }
#pragma unroll
    for (int j = 0; j < 2 * R; ++j) cc[j] = j < cnt ? c[j] : INT_MAX;
#pragma unroll
    for (int i = 0; i < R; ++i) {
      if (ww[i] < v) {
        int rk = 0;
#pragma unroll
        for (int j = 0; j < 2 * R; ++j) rk += cc[j] < ww[i];
        const int e = base + rk, h = hh[i], tw = twin[h];
        eid[h] = e;
        e2h[e] = (tw >= 0 && tw < h) ? tw : h;
        bflag[e] = tw < 0;
        nb += tw < 0;
      }
      if (uu[i] < v) {
        int rk = 0;
#pragma unroll
        for (int j = 0; j < 2 * R; ++j) rk += cc[j] < uu[i];
        const int e = base + rk, hp = pv[i];
        eid[hp] = e;
        if (twin[hp] < 0) {  // boundary edge u->v with no half-edge v->u
          e2h[e] = hp;
          bflag[e] = 1;
          ++nb;
        }
      }
    }
  } else {
    for (int i = 0; i < n; ++i) {
      const int h = inc[r0 + i];
      const int w = t.fv[he_next<ORDER>(t, h)];
      if (w < v) {
        const int e = base + rank_of(c, cnt, w);
        eid[h] = e;
        const int tw = twin[h];
        e2h[e] = (tw >= 0 && tw < h) ? tw : h;
        bflag[e] = tw < 0;
        nb += tw < 0;
      }
      const int hp = he_prev<ORDER>(t, h);
      const int u = t.fv[hp];
      if (u < v) {
        const int e = base + rank_of(c, cnt, u);
        eid[hp] = e;
        if (twin[hp] < 0) {  // boundary edge u->v with no half-edge v->u
          e2h[e] = hp;
          bflag[e] = 1;
          ++nb;
        }
      }
    }
  }
  if (nb) atomicAdd(&info->num_boundary, nb);
}

hipError_t build_faces(const Topo &t, int scheme, const BuildScratch &b, DeviceInfo *info, hipStream_t s,
                       bool cleared) {
  hipError_t err;
  if (!cleared) {
    ZeroRegions z{};
    z.p[0] = b.nval;
    z.n[0] = t.V + 1ll;
    z.p[1] = b.cursor;
    z.n[1] = t.V;
    z.count = 2;
    if ((err = launch_zero_regions(z, s)) != hipSuccess) return err;
  }
  const unsigned gf = grid_for(t.F);
  if (t.order == 4)
    hipLaunchKernelGGL(k_build_faces<4>, dim3(gf), dim3(kBlock), 0, s, t, scheme, b.nval, (int32_t *)nullptr, info);
  else if (t.order == 3)
    hipLaunchKernelGGL(k_build_faces<3>, dim3(gf), dim3(kBlock), 0, s, t, scheme, b.nval, (int32_t *)nullptr, info);
  else
    hipLaunchKernelGGL(k_build_faces<0>, dim3(gf), dim3(kBlock), 0, s, t, scheme, b.nval,
                       const_cast<int32_t *>(t.hface), info);
  return hipGetLastError();
}

hipError_t build_adjacency(const Topo &t, int scheme, const BuildScratch &b, Adj &a, DeviceInfo *info,
                           hipStream_t s) {
  (void)scheme;
  hipError_t err;
  if ((err = launch_scan(b.nval, b.rowptr, t.V, b.partials, nullptr, s)) != hipSuccess) return err;
  hipLaunchKernelGGL(k_build_incidence, dim3(grid_for(t.H)), dim3(kBlock), 0, s, t, (const int32_t *)b.rowptr,
                     b.cursor, b.inc, (const DeviceInfo *)info);
  if ((err = hipGetLastError()) != hipSuccess) return err;
  const unsigned gv = grid_for(t.V);
  if (t.order == 4)
    hipLaunchKernelGGL(k_build_vertex<4>, dim3(gv), dim3(kBlock), 0, s, t, (const int32_t *)b.rowptr, b.inc, b.cand,
                       a.twin, a.vhe, b.cntlo, info);
  else if (t.order == 3)
    hipLaunchKernelGGL(k_build_vertex<3>, dim3(gv), dim3(kBlock), 0, s, t, (const int32_t *)b.rowptr, b.inc, b.cand,
                       a.twin, a.vhe, b.cntlo, info);
  else
    hipLaunchKernelGGL(k_build_vertex<0>, dim3(gv), dim3(kBlock), 0, s, t, (const int32_t *)b.rowptr, b.inc, b.cand,
                       a.twin, a.vhe, b.cntlo, info);
  if ((err = hipGetLastError()) != hipSuccess) return err;
  if ((err = launch_scan(b.cntlo, b.ebase, t.V, b.partials, &info->num_edges, s)) != hipSuccess) return err;
#define SUBDIV_EID_ARGS                                                                                        \
  t, (const int32_t *)b.rowptr, (const int32_t *)b.inc, (const int32_t *)b.cand, (const int32_t *)b.cntlo,     \
      (const int32_t *)b.ebase, (const int32_t *)a.twin, a.eid, a.e2h, b.bflag, info
  if (t.order == 4)
    hipLaunchKernelGGL(k_build_eid<4>, dim3(gv), dim3(kBlock), 0, s, SUBDIV_EID_ARGS);
  else if (t.order == 3)
    hipLaunchKernelGGL(k_build_eid<3>, dim3(gv), dim3(kBlock), 0, s, SUBDIV_EID_ARGS);
  else
    hipLaunchKernelGGL(k_build_eid<0>, dim3(gv), dim3(kBlock), 0, s, SUBDIV_EID_ARGS);
#undef SUBDIV_EID_ARGS
  return hipGetLastError();
}

hipError_t build_bscan(const Topo &t, const BuildScratch &b, Adj &a, hipStream_t s) {
  (void)t;
  return launch_scan(b.bflag, a.bscan, a.E, b.partials, nullptr, s);
}

// crease matrix C (Sec. 3.3) placed on edge ids: sig[eid] = sigma
// the crease matrix C placed onto edge ids: edge (lo, hi) is
// ebase[hi] + rank of lo among hi's sorted lower neighbours
__global__ void k_build_creases(Topo t, const int32_t *rowptr, const int32_t *cand, const int32_t *cntlo,
                                const int32_t *ebase, int C, const int32_t *cv, const float *cs, double *sig,
                                int32_t *sigcnt, DeviceInfo *info) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= C || faulted(info)) return;
  const int a = cv[2 * i], b = cv[2 * i + 1];
  const float s = cs[i];
  if (a < 0 || a >= t.V || b < 0 || b >= t.V || a == b || !(s >= 0.0f) || isinf(s)) {
    atomicOr(&info->faults, FAULT_BAD_CREASE);
    return;
  }
  if (s == 0.0f) return;  // a smooth edge
  const int hi = a > b ? a : b, lo = a > b ? b : a;
  const int32_t *c = cand + 2 * rowptr[hi];
  const int n = cntlo[hi], r = rank_of(c, n, lo);
  const int e = (r < n && c[r] == lo) ? ebase[hi] + r : -1;
  if (e < 0 || atomicAdd(&sigcnt[e], 1) != 0) {
    atomicOr(&info->faults, FAULT_BAD_CREASE);
    return;
  }
  sig[e] = (double)s;
  atomicMax(&info->max_sharp_bits, __float_as_uint(s));
}

// Two triangles on the same three vertices with opposite orientations are a
// closed two-face component; refining it by Loop or sqrt(3) gives a level on
// which edges are shared by more than two faces.
__global__ void k_count_pillows(Topo t, const int32_t *twin, DeviceInfo *info) {
  const int f = blockIdx.x * blockDim.x + threadIdx.x;
  if (f >= t.F || faulted(info)) return;
  const int a = twin[3 * f], b = twin[3 * f + 1], c = twin[3 * f + 2];
  if (a >= 0 && b >= 0 && c >= 0 && a / 3 == b / 3 && b / 3 == c / 3) atomicAdd(&info->num_pillows, 1);
}

hipError_t count_pillows(const Topo &t, const Adj &a, DeviceInfo *info, hipStream_t s) {
  hipLaunchKernelGGL(k_count_pillows, dim3(grid_for(t.F)), dim3(kBlock), 0, s, t, (const int32_t *)a.twin, info);
  return hipGetLastError();
}

hipError_t build_creases(const Topo &t, const BuildScratch &b, const Adj &a, int C, const int32_t *cv,
                         const float *cs, DeviceInfo *info, hipStream_t s) {
  if (C <= 0) return hipSuccess;
  hipLaunchKernelGGL(k_build_creases, dim3(grid_for(C)), dim3(kBlock), 0, s, t, (const int32_t *)b.rowptr,
                     (const int32_t *)b.cand, (const int32_t *)b.cntlo, (const int32_t *)b.ebase, C, cv, cs, a.sig,
                     b.sigcnt, info);
  return hipGetLastError();
}

// (lo, hi) of every edge in id order
template <int ORDER>
__global__ void k_edge_export(Topo t, const int32_t *e2h, int E, int32_t *out) {
  const int e = blockIdx.x * blockDim.x + threadIdx.x;
  if (e >= E) return;
  const int h = e2h[e];
  const int a = t.fv[h], b = t.fv[he_next<ORDER>(t, h)];
  out[2 * e] = a < b ? a : b;
  out[2 * e + 1] = a < b ? b : a;
}

hipError_t launch_edge_export(const Topo &t, const Adj &a, int32_t *out, hipStream_t s) {
  if (t.order == 4)
    hipLaunchKernelGGL(k_edge_export<4>, dim3(grid_for(a.E)), dim3(kBlock), 0, s, t, (const int32_t *)a.e2h, a.E,
                       out);
  else if (t.order == 3)
    hipLaunchKernelGGL(k_edge_export<3>, dim3(grid_for(a.E)), dim3(kBlock), 0, s, t, (const int32_t *)a.e2h, a.E,
                       out);
  else
    hipLaunchKernelGGL(k_edge_export<0>, dim3(grid_for(a.E)), dim3(kBlock), 0, s, t, (const int32_t *)a.e2h, a.E,
                       out);
  return hipGetLastError();
}

}  // namespace subdiv
