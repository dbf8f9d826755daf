// Batched refinement of uneven meshes on gfx950: the meshes of a batch are
// packed into one disjoint union cage (vertex, face, half-edge and crease
// offsets), the union is refined by the ordinary per-level kernels -- one
// launch per stage for the whole batch -- and every mesh's final level is
// then gathered into its own buffers in its own local numbering.
//
// Why this gives every mesh exactly its solo result: the refinement of a
// disjoint union is the union of the refinements, and the union's index
// rules keep each mesh's elements in their relative order. A refined level
// lists [vertex points | face points | edge points] (Catmull-Clark; Loop
// has no face block, sqrt(3) no edge block); inside each block the meshes
// appear one after the other, each in its own order, because faces stay
// grouped by mesh (children of face r sit at col_ptr[r] + j) and edges stay
// grouped by mesh (every edge of a refined Catmull-Clark or Loop level has
// an edge point as its higher end, and the upper triangle of E is
// enumerated by that end). Ranks within a mesh are unchanged, so the
// arithmetic on every element is the same as when the mesh is refined alone.
#include "subdiv_internal.h"

namespace subdiv {

__device__ __forceinline__ int seg_of(const int32_t *pre, int n, int x) {
  // largest i in [0, n) with pre[i] <= x
  int lo = 0, hi = n;
  while (hi - lo > 1) {
    const int mid = (lo + hi) >> 1;
    if (pre[mid] <= x) lo = mid;
    else hi = mid;
  }
  return lo;
}

// ---- pack the cages into the union (topology and creases) ---------------
__global__ void k_concat_topology(const BatchMesh *m, int n, BatchUnion u) {
  const long long gid = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  const int total_h = m[n - 1].hofs + m[n - 1].H;
  const int total_f = m[n - 1].fofs + m[n - 1].F;
  const int total_c = m[n - 1].cofs + m[n - 1].C;
  if (gid < total_h) {
    int lo = 0, hi = n;
    while (hi - lo > 1) {
      const int mid = (lo + hi) >> 1;
      if (m[mid].hofs <= gid) lo = mid;
      else hi = mid;
    }
    const BatchMesh &b = m[lo];
    u.fv[gid] = b.fv[gid - b.hofs] + b.vofs;
  }
  if (u.off && gid <= total_f) {
    if (gid == total_f) {
      u.off[gid] = total_h;
    } else {
      int lo = 0, hi = n;
      while (hi - lo > 1) {
        const int mid = (lo + hi) >> 1;
        if (m[mid].fofs <= gid) lo = mid;
        else hi = mid;
      }
      const BatchMesh &b = m[lo];
      const int f = (int)gid - b.fofs;
      u.off[gid] = b.hofs + (b.off ? b.off[f] : f * b.order);
    }
  }
  if (gid < total_c) {
    int lo = 0, hi = n;
    while (hi - lo > 1) {
      const int mid = (lo + hi) >> 1;
      if (m[mid].cofs <= gid) lo = mid;
      else hi = mid;
    }
    const BatchMesh &b = m[lo];
    const int c = (int)gid - b.cofs;
    u.cv[2 * gid] = b.cv[2 * c] + b.vofs;
    u.cv[2 * gid + 1] = b.cv[2 * c + 1] + b.vofs;
    u.cs[gid] = b.cs[c];
  }
}

__global__ void k_concat_positions(const BatchMesh *m, int n, float *P) {
  const int gid = blockIdx.x * blockDim.x + threadIdx.x;
  const int total_v = m[n - 1].vofs + m[n - 1].V;
  if (gid >= total_v) return;
  int lo = 0, hi = n;
  while (hi - lo > 1) {
    const int mid = (lo + hi) >> 1;
    if (m[mid].vofs <= gid) lo = mid;
    else hi = mid;
  }
  const BatchMesh &b = m[lo];
  st3(P, gid, ld3(b.P, gid - b.vofs));
}

// ---- per-mesh counts of the union cage ---------------------------------
// ebase = exclusive scan of lower-neighbour counts (edge base per vertex);
// the edges of mesh i are ebase[vofs_i] .. ebase[vofs_{i+1}]
__global__ void k_batch_edge_ranges(const BatchMesh *m, int n, const int32_t *ebase, int32_t *epre) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i > n) return;
  const int v = (i == n) ? m[n - 1].vofs + m[n - 1].V : m[i].vofs;
  epre[i] = ebase[v];
}

// boundary edges per mesh (the grid covers an upper bound of the union's
// edges; the scan total epre[n] is the count)
__global__ void k_batch_boundary_counts(const int32_t *epre, int n, const int32_t *bflag, int32_t *bcount) {
  const int e = blockIdx.x * blockDim.x + threadIdx.x;
  if (e >= epre[n]) return;
  if (bflag[e]) atomicAdd(&bcount[seg_of(epre, n + 1, e)], 1);
}

// largest valence (incident faces, from the row pointer of M's row view) and
// largest crease sharpness (float bits: sharpness is validated >= 0, so the
// bits order like the values) per mesh
__global__ void k_batch_maxima(const BatchMesh *m, int n, const int32_t *rowptr, const float *cs, long long VU,
                               long long CU, int32_t *vmax, int32_t *smax) {
  const long long gid = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  if (gid < VU) {
    int lo = 0, hi = n;
    while (hi - lo > 1) {
      const int mid = (lo + hi) >> 1;
      if (m[mid].vofs <= gid) lo = mid;
      else hi = mid;
    }
    atomicMax(&vmax[lo], rowptr[gid + 1] - rowptr[gid]);
  }
  if (gid < CU) {
    int lo = 0, hi = n;
    while (hi - lo > 1) {
      const int mid = (lo + hi) >> 1;
      if (m[mid].cofs <= gid) lo = mid;
      else hi = mid;
    }
    atomicMax(&smax[lo], __float_as_int(cs[gid]));
  }
}

// ---- gather the union's final level into each mesh's buffers ----------
// Both gathers give every workgroup one chunk of kGather elements of one
// segment, found by a binary search over the chunk prefix; inside the chunk
// the copy is contiguous on both sides.
// faces: the union faces of mesh i are contiguous; a corner u lies in block
// b = the last block starting at or below u, and its local id is u + doff(b, i)
__global__ void __launch_bounds__(kBlock) k_extract_faces(BatchTables t, const int32_t *fvL, const BatchOut *out) {
  const int c = blockIdx.x;
  const int i = seg_of(t.fch, t.n, c);
  const long long f0 = (long long)t.fpre[i] + (long long)(c - t.fch[i]) * kGather;
  const long long f1 = min(f0 + kGather, (long long)t.fpre[i + 1]);
  const long long x0 = t.order * f0, x1 = t.order * f1, base = (long long)t.order * t.fpre[i];
  const int32_t *doff = t.doff + i;
  int32_t *dst = out[i].fv;
  for (long long x = x0 + threadIdx.x; x < x1; x += blockDim.x) {
    const int u = fvL[x];
    dst[x - base] = u + doff[(long long)seg_of(t.ub, t.nblk, u) * t.n];
  }
}

// positions: segment (block b, mesh i) is one contiguous run on both sides
__global__ void __launch_bounds__(kBlock) k_extract_positions(BatchTables t, const float *PL, const BatchOut *out) {
  const int c = blockIdx.x;
  const int sidx = seg_of(t.pch, t.nseg, c);
  const int4 g = t.seg[sidx];  // (union start, mesh, local start, length)
  const long long e0 = (long long)(c - t.pch[sidx]) * kGather;
  const long long e1 = min(e0 + kGather, (long long)g.w);
  const float *src = PL + 3ll * (g.x + e0);
  float *dst = out[g.y].P + 3ll * (g.z + e0);
  for (long long x = threadIdx.x; x < 3 * (e1 - e0); x += blockDim.x) dst[x] = src[x];
}

hipError_t batch_concat_topology(const BatchMesh *m, int n, const BatchUnion &u, long long items, hipStream_t s) {
  hipLaunchKernelGGL(k_concat_topology, dim3(grid_for(items)), dim3(kBlock), 0, s, m, n, u);
  return hipGetLastError();
}

hipError_t batch_concat_positions(const BatchMesh *m, int n, float *P, long long V, hipStream_t s) {
  hipLaunchKernelGGL(k_concat_positions, dim3(grid_for(V)), dim3(kBlock), 0, s, m, n, P);
  return hipGetLastError();
}

hipError_t batch_stats(const BatchMesh *m, int n, const int32_t *ebase, const int32_t *bflag, const int32_t *rowptr,
                       const float *cs, long long VU, long long HU, long long CU, int32_t *epre, int32_t *bcount,
                       int32_t *vmax, int32_t *smax, hipStream_t s) {
  // bcount, vmax and smax are consecutive: one fill clears all three
  hipError_t err = launch_fill_i32(bcount, 0, 3ll * n, s);
  if (err != hipSuccess) return err;
  hipLaunchKernelGGL(k_batch_edge_ranges, dim3(grid_for(n + 1)), dim3(kBlock), 0, s, m, n, ebase, epre);
  hipLaunchKernelGGL(k_batch_boundary_counts, dim3(grid_for(HU)), dim3(kBlock), 0, s, (const int32_t *)epre, n, bflag,
                     bcount);
  const long long items = VU > CU ? VU : CU;
  hipLaunchKernelGGL(k_batch_maxima, dim3(grid_for(items)), dim3(kBlock), 0, s, m, n, rowptr, cs, VU, CU, vmax, smax);
  return hipGetLastError();
}

hipError_t batch_extract(const BatchTables &t, const int32_t *fvL, const float *PL, const BatchOut *out,
                         int face_chunks, int vertex_chunks, hipStream_t s) {
  if (face_chunks > 0)
    hipLaunchKernelGGL(k_extract_faces, dim3(face_chunks), dim3(kBlock), 0, s, t, fvL, out);
  if (vertex_chunks > 0)
    hipLaunchKernelGGL(k_extract_positions, dim3(vertex_chunks), dim3(kBlock), 0, s, t, PL, out);
  return hipGetLastError();
}

}  // namespace subdiv
