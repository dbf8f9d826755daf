// Selective subdivision's extraction step on gfx950 (Sec. 3.4): the region
// around selected vertices is cut out of a cage as a cage of its own, which
// is then planned and refined like any other.
//
//   x_0     selected vertices: a caller's mask, or the extraordinary ones
//           (valence n = M 1 of eq:vo, the incident faces, not four);
//   q_i     = M^T x_i: faces with a selected corner (one lane per face);
//   x_{i+1} = M q_i: the corners of those faces (one lane per face marks
//           them; every lane writes the same 1, so the result does not depend
//           on which lane writes last);
//   M'      = X M X-ring, P' = X P: X and X-ring are identities with the rows
//           of unselected vertices / columns of unselected faces deleted, so
//           the survivors keep their order and their new ids are exclusive
//           scans of the flags; a face keeps its corners in cyclic order.
// Creases of the cage whose edge is an edge of an extracted face are kept,
// emitted once from the lower selected half-edge of the edge.
#include "subdiv_internal.h"

namespace subdiv {

__global__ void k_sel_seed(int V, const uint8_t *seed, const int32_t *valence, int32_t *x, uint8_t *x0) {
  const int v = blockIdx.x * blockDim.x + threadIdx.x;
  if (v >= V) return;
  const int s = seed ? (seed[v] != 0) : (valence[v] != 4);
  x[v] = s;
  x0[v] = (uint8_t)s;  // kept for the extraction's seed flags (x[] is overwritten by later rings)
}

template <int ORDER>
__global__ void k_sel_faces(Topo t, const int32_t *x, int32_t *q) {
  const int f = blockIdx.x * blockDim.x + threadIdx.x;
  if (f >= t.F) return;
  int any = 0;
  for (int h = face_begin<ORDER>(t, f); h < face_end<ORDER>(t, f); ++h) any |= x[t.fv[h]];
  q[f] = any;
}

template <int ORDER>
__global__ void k_sel_mark(Topo t, const int32_t *q, int32_t *x) {
  const int f = blockIdx.x * blockDim.x + threadIdx.x;
  if (f >= t.F || !q[f]) return;
  for (int h = face_begin<ORDER>(t, f); h < face_end<ORDER>(t, f); ++h) x[t.fv[h]] = 1;
}

// Pinch closing (a reading; the paper's extraction matrices do not meet the
// case): two selected regions that touch at one vertex would give the
// extraction a vertex with two fans, which is no manifold. Per pass, every
// selected vertex whose selected faces around it form more than one run in
// rotation order marks its whole star (into qadd: the pass reads q alone, so
// the result does not depend on lane order); the merge then adds those faces
// to q and their corners to x. A pass whose predecessor changed nothing does
// nothing.
template <int ORDER>
__global__ void k_pinch_find(Topo t, Adj a, const int32_t *q, const int32_t *x, int32_t *qadd, int32_t *changed,
                             int pass) {
  const int v = blockIdx.x * blockDim.x + threadIdx.x;
  if (v >= t.V || !x[v] || (pass > 0 && changed[pass - 1] == 0)) return;
  const int h0 = a.vhe[v];
  int runs = 0, first = -1, prev = -1, n = 0;
  int h = h0;
  while (true) {
    const int sel = q[he_face<ORDER>(t, h)] != 0;
    if (n == 0) first = sel;
    else runs += (sel && !prev);
    prev = sel;
    ++n;
    const int tw = a.twin[he_prev<ORDER>(t, h)];
    if (tw < 0) {  // the fan ends at the boundary: the first run starts at the first face
      runs += first;
      break;
    }
    if (tw == h0 || n >= SUBDIV_MAX_VALENCE) {  // closed: the first face follows the last
      runs += (first && !prev);
      if (runs == 0 && first) runs = 1;  // the whole star
      break;
    }
    h = tw;
  }
  if (runs < 2) return;
  h = h0;
  for (int i = 0; i < n; ++i) {
    qadd[he_face<ORDER>(t, h)] = 1;
    const int tw = a.twin[he_prev<ORDER>(t, h)];
    if (tw < 0) break;
    h = tw;
  }
  changed[pass] = 1;
}

template <int ORDER>
__global__ void k_pinch_merge(Topo t, int32_t *q, int32_t *x, const int32_t *qadd, const int32_t *changed, int pass) {
  const int f = blockIdx.x * blockDim.x + threadIdx.x;
  if (f >= t.F || changed[pass] == 0 || !qadd[f]) return;
  q[f] = 1;
  for (int h = face_begin<ORDER>(t, f); h < face_end<ORDER>(t, f); ++h) x[t.fv[h]] = 1;
}

// corners of the selected faces (for the column pointer of a general cage)
template <int ORDER>
__global__ void k_sel_sizes(Topo t, const int32_t *q, int32_t *sizes) {
  const int f = blockIdx.x * blockDim.x + threadIdx.x;
  if (f >= t.F) return;
  sizes[f] = q[f] ? face_end<ORDER>(t, f) - face_begin<ORDER>(t, f) : 0;
}

// half-edges that emit a crease: in a selected face, on a sharp edge, and the
// lower of the edge's selected half-edges
template <int ORDER>
__global__ void k_sel_creases(Topo t, Adj a, const int32_t *q, int32_t *flag) {
  const int h = blockIdx.x * blockDim.x + threadIdx.x;
  if (h >= t.H) return;
  int emit = 0;
  if (q[he_face<ORDER>(t, h)] && a.sig[a.eid[h]] > 0.0) {
    const int tw = a.twin[h];
    emit = (tw < 0 || !q[he_face<ORDER>(t, tw)] || h < tw);
  }
  flag[h] = emit;
}

__global__ void k_ext_vertices(int V, const int32_t *x, const int32_t *vnew, const float *P, float *P1,
                               int32_t *vmap, const uint8_t *x0, uint8_t *seed1) {
  const int v = blockIdx.x * blockDim.x + threadIdx.x;
  if (v >= V || !x[v]) return;
  const int n = vnew[v];
  st3(P1, n, ld3(P, v));
  if (vmap) vmap[n] = v;
  if (seed1) seed1[n] = x0[v];
}

template <int ORDER>
__global__ void k_ext_faces(Topo t, const int32_t *q, const int32_t *fnew, const int32_t *onew,
                            const int32_t *vnew, int32_t *fv1, int32_t *off1, int32_t *fmap, int F1) {
  const int f = blockIdx.x * blockDim.x + threadIdx.x;
  if (f >= t.F || !q[f]) return;
  const int n = fnew[f];
  const int b = face_begin<ORDER>(t, f), en = face_end<ORDER>(t, f);
  const int o = ORDER > 0 ? ORDER * n : onew[f];
  for (int h = b; h < en; ++h) fv1[o + (h - b)] = vnew[t.fv[h]];
  if (ORDER == 0) {
    off1[n] = o;
    if (n == F1 - 1) off1[F1] = o + (en - b);
  }
  if (fmap) fmap[n] = f;
}

template <int ORDER>
__global__ void k_ext_creases(Topo t, Adj a, const int32_t *flag, const int32_t *cnew, const int32_t *vnew,
                              int32_t *cv1, float *cs1) {
  const int h = blockIdx.x * blockDim.x + threadIdx.x;
  if (h >= t.H || !flag[h]) return;
  const int c = cnew[h];
  cv1[2 * c] = vnew[t.fv[h]];
  cv1[2 * c + 1] = vnew[t.fv[he_next<ORDER>(t, h)]];
  cs1[c] = (float)a.sig[a.eid[h]];  // the cage's FP32 sharpness, held exactly in FP64
}

template <int ORDER>
static hipError_t select_t(const Topo &t, const Adj &a, const SelectScratch &w, const uint8_t *seed,
                           const int32_t *valence, int rings, bool close_pinches, hipStream_t s) {
  hipError_t err;
  const unsigned gv = grid_for(t.V), gf = grid_for(t.F), gh = grid_for(t.H);
  int32_t *x = w.x[0], *xn = w.x[1];
  hipLaunchKernelGGL(k_sel_seed, dim3(gv), dim3(kBlock), 0, s, t.V, seed, valence, x, w.seed0);
  for (int i = 0; i < rings; ++i) {
    hipLaunchKernelGGL(k_sel_faces<ORDER>, dim3(gf), dim3(kBlock), 0, s, t, x, w.q);
    if ((err = launch_fill_i32(xn, 0, t.V, s)) != hipSuccess) return err;
    hipLaunchKernelGGL(k_sel_mark<ORDER>, dim3(gf), dim3(kBlock), 0, s, t, w.q, xn);
    int32_t *tmp = x;
    x = xn;
    xn = tmp;
  }
  // the final vertex flags always sit in x[rings & 1]
  if (close_pinches) {
    if ((err = launch_fill_i32(w.qadd, 0, t.F, s)) != hipSuccess) return err;
    if ((err = launch_fill_i32(w.changed, 0, kPinchPasses, s)) != hipSuccess) return err;
    for (int p = 0; p < kPinchPasses; ++p) {
      hipLaunchKernelGGL(k_pinch_find<ORDER>, dim3(gv), dim3(kBlock), 0, s, t, a, w.q, x, w.qadd, w.changed, p);
      hipLaunchKernelGGL(k_pinch_merge<ORDER>, dim3(gf), dim3(kBlock), 0, s, t, w.q, x, w.qadd, w.changed, p);
    }
  }
  if ((err = launch_scan(x, w.vnew, t.V, w.partials, w.totals + 0, s)) != hipSuccess) return err;
  if ((err = launch_scan(w.q, w.fnew, t.F, w.partials, w.totals + 1, s)) != hipSuccess) return err;
  if (ORDER == 0) {
    hipLaunchKernelGGL(k_sel_sizes<ORDER>, dim3(gf), dim3(kBlock), 0, s, t, w.q, w.flag);
    if ((err = launch_scan(w.flag, w.onew, t.F, w.partials, w.totals + 2, s)) != hipSuccess) return err;
  }
  if (a.sig) {
    hipLaunchKernelGGL(k_sel_creases<ORDER>, dim3(gh), dim3(kBlock), 0, s, t, a, w.q, w.flag);
    if ((err = launch_scan(w.flag, w.cnew, t.H, w.partials, w.totals + 3, s)) != hipSuccess) return err;
  } else if ((err = launch_fill_i32(w.totals + 3, 0, 1, s)) != hipSuccess) {
    return err;
  }
  return hipGetLastError();
}

hipError_t select_region(const Topo &t, const Adj &a, const SelectScratch &w, const uint8_t *seed,
                         const int32_t *valence, int rings, bool close_pinches, hipStream_t s) {
  if (t.order == 4) return select_t<4>(t, a, w, seed, valence, rings, close_pinches, s);
  if (t.order == 3) return select_t<3>(t, a, w, seed, valence, rings, close_pinches, s);
  return select_t<0>(t, a, w, seed, valence, rings, close_pinches, s);
}

template <int ORDER>
static hipError_t extract_t(const Topo &t, const Adj &a, const SelectScratch &w, int rings, const float *P,
                            const ExtractOut &o, hipStream_t s) {
  const int32_t *x = w.x[rings & 1];
  hipLaunchKernelGGL(k_ext_vertices, dim3(grid_for(t.V)), dim3(kBlock), 0, s, t.V, x, w.vnew, P, o.P, o.vmap,
                     (const uint8_t *)w.seed0, o.seed);
  hipLaunchKernelGGL(k_ext_faces<ORDER>, dim3(grid_for(t.F)), dim3(kBlock), 0, s, t, w.q, w.fnew, w.onew, w.vnew,
                     o.fv, o.off, o.fmap, o.F);
  if (a.sig && o.C > 0) {
    // crease flags again (cheap), so that nothing between the two calls matters
    hipLaunchKernelGGL(k_sel_creases<ORDER>, dim3(grid_for(t.H)), dim3(kBlock), 0, s, t, a, w.q, w.flag);
    hipLaunchKernelGGL(k_ext_creases<ORDER>, dim3(grid_for(t.H)), dim3(kBlock), 0, s, t, a, w.flag, w.cnew, w.vnew,
                       o.cv, o.cs);
  }
  return hipGetLastError();
}

hipError_t extract_region(const Topo &t, const Adj &a, const SelectScratch &w, int rings, const float *P,
                          const ExtractOut &o, hipStream_t s) {
  if (t.order == 4) return extract_t<4>(t, a, w, rings, P, o, s);
  if (t.order == 3) return extract_t<3>(t, a, w, rings, P, o, s);
  return extract_t<0>(t, a, w, rings, P, o, s);
}

}  // namespace subdiv
