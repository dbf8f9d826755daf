// One Catmull-Clark level on gfx950 from the adjacency of the same level:
// the cage step, and every step when levels are rebuilt on request. Eval
// (face, edge and vertex points, boundary repair, creases), the face table
// of the next level and the inherited sharpness of its edges.
//
// Rules (Sec. 3.1 / 3.2): face point f_r = mapped M^T P (eq:spla_fp); edge
// point 1/4 (p_k + p_l + f_r + f_s) with f_r, f_s = F(k,l), F(l,k) (eq:F);
// vertex update s1 + s2 + s3 = (1 - 2/n) p + 1/n^2 sum p_j + 1/n^2 sum f_j with
// n = M 1 (eq:vo); boundary repair (eq::CC_boundary); creases overwrite the
// smooth values (Sec. 3.3, fig. module_creases) and are inherited with the
// Chaikin-type sharpness rule.
//
// Topology of level k+1 (Sec. 3.2 "Topology refinement"): child j of face r
// is (v_j, |v|+|f|+e(v_j,v_j+1), |v|+r, |v|+|f|+e(v_j-1,v_j)) at index
// col_ptr[r] + j, i.e. child index == parent half-edge index h. Every edge of
// level k+1 has an edge point as its higher end, so its lower neighbours are,
// ascending, lo(e), hi(e), then the face points of the (one or two) faces of
// e: the children of edge e have ids base(e) + rank, base(e) = 4 e -
// (boundary edges before e). The next level's own adjacency is carried over
// in closed form by the parent-level kernels (cc_lag.hip).
#include "subdiv_internal.h"

namespace subdiv {

__device__ __forceinline__ double chaikin(double si, double sj) {
  // max(1/4 (si + 3 sj) - 1, 0) in this exact operation order; the pragma keeps
  // the compiler from fusing a product and a sum (HIP's __dadd_rn and
  // __dmul_rn are plain operators, which it may contract)
#pragma clang fp contract(off)
  const double t = 0.25 * (si + 3.0 * sj) - 1.0;
  return t > 0.0 ? t : 0.0;
}

__device__ __forceinline__ int edge_base(const CCStep &c, int e) {
  return 4 * e - (c.has_bnd ? c.a.bscan[e] : 0);
}

// ---------------------------------------------------------------- faces
template <int ORDER>
__global__ void __launch_bounds__(kBlock) k_cc_face(CCStep c) {
  const int r = blockIdx.x * blockDim.x + threadIdx.x;
  if (r >= c.t.F) return;
  const int V = c.t.V, F = c.t.F;
  const int VF = V + F;
  if constexpr (ORDER == 4) {
    const int4 q = reinterpret_cast<const int4 *>(c.t.fv)[r];
    const int4 ed = reinterpret_cast<const int4 *>(c.a.eid)[r];
    const int v[4] = {q.x, q.y, q.z, q.w};
    const int e[4] = {ed.x, ed.y, ed.z, ed.w};
    const f3 p0 = ld3(c.P, v[0]), p1 = ld3(c.P, v[1]), p2 = ld3(c.P, v[2]), p3 = ld3(c.P, v[3]);
    // summed in slot order, as the general-polygon path does, so a quad cage
    // gives the same bits whether or not it comes with a column pointer
    st3(c.P1, V + r, mul3(0.25f, add3(add3(add3(p0, p1), p2), p3)));
    if (c.fv1) {
      int4 *out = reinterpret_cast<int4 *>(c.fv1) + 4ll * r;
#pragma unroll
      for (int j = 0; j < 4; ++j) out[j] = make_int4(v[j], VF + e[j], V + r, VF + e[(j + 3) & 3]);
    }
  } else {
    // general polygons (a cage with a column pointer) and triangle cages
    const int b = face_begin<ORDER>(c.t, r), en = face_end<ORDER>(c.t, r), n = en - b;
    f3 acc{0.f, 0.f, 0.f};
    for (int h = b; h < en; ++h) acc = add3(acc, ld3(c.P, c.t.fv[h]));
    st3(c.P1, V + r, mul3(1.0f / (float)n, acc));
    if (c.fv1)
      for (int h = b; h < en; ++h) {
        const int hp = (h == b) ? en - 1 : h - 1;
        reinterpret_cast<int4 *>(c.fv1)[h] = make_int4(c.t.fv[h], VF + c.a.eid[h], V + r, VF + c.a.eid[hp]);
      }
  }
}

// ---------------------------------------------------------------- vertices
template <int ORDER>
__global__ void __launch_bounds__(kBlock) k_cc_vertex(CCStep c) {
  const int v = blockIdx.x * blockDim.x + threadIdx.x;
  if (v >= c.t.V) return;
  const int V = c.t.V;
  const int h0 = c.a.vhe[v];
  const f3 p = ld3(c.P, v);
  const bool bnd = c.a.twin[h0] < 0;
  f3 sp{0.f, 0.f, 0.f}, sf{0.f, 0.f, 0.f};
  int n = 0, k = 0, cv0 = -1, cv1 = -1, ce0 = -1, ce1 = -1, ub = -1;
  double ssum = 0.0;
  int h = h0;
  while (true) {
    const int w = c.t.fv[he_next<ORDER>(c.t, h)];
    sp = add3(sp, ld3(c.P, w));
    sf = add3(sf, ld3(c.P1, V + he_face<ORDER>(c.t, h)));
    ++n;
    if (c.creases) {
      const int e = c.a.eid[h];
      const double s = c.a.sig[e];
      if (s > 0.0) {
        if (k == 0) { cv0 = w; ce0 = e; } else if (k == 1) { cv1 = w; ce1 = e; }
        ++k;
        ssum += s;
      }
    }
    const int hp = he_prev<ORDER>(c.t, h);
    const int t = c.a.twin[hp];
    if (t < 0) {
      ub = c.t.fv[hp];
      if (c.creases) {
        const int e = c.a.eid[hp];
        const double s = c.a.sig[e];
        if (s > 0.0) {
          if (k == 0) { cv0 = ub; ce0 = e; } else if (k == 1) { cv1 = ub; ce1 = e; }
          ++k;
          ssum += s;
        }
      }
      break;
    }
    if (t == h0 || n >= SUBDIV_MAX_VALENCE) break;
    h = t;
  }
  f3 S;
  if (bnd) {  // eq::CC_boundary: 3/4 p + 1/8 (p_prev + p_next)
    const int w0 = c.t.fv[he_next<ORDER>(c.t, h0)];
    S = fma3(0.75f, p, mul3(0.125f, add3(ld3(c.P, w0), ld3(c.P, ub))));
  } else {
    const float fn = (float)n;
    const float inv2 = 1.0f / (fn * fn);
    S = fma3(1.0f - 2.0f / fn, p, mul3(inv2, add3(sp, sf)));
    if (c.creases && k >= 2) {
      const f3 sharp = (k == 2) ? fma3(0.75f, p, mul3(0.125f, add3(ld3(c.P, cv0), ld3(c.P, cv1)))) : p;
      const double s = ssum / (double)k;
      if (s >= 1.0) S = sharp;
      else {
        const float fs = (float)s;
        S = fma3(1.0f - fs, S, mul3(fs, sharp));
      }
    }
  }
  st3(c.P1, v, S);
  if (c.creases) c.a.vcr[v] = make_int4(k, ce0, ce1, 0);
}

// ---------------------------------------------------------------- edges
template <int ORDER>
__global__ void __launch_bounds__(kBlock) k_cc_edge(CCStep c) {
  const int e = blockIdx.x * blockDim.x + threadIdx.x;
  if (e >= c.a.E) return;
  const int V = c.t.V, F = c.t.F;
  const int h = c.a.e2h[e];
  const int hn = he_next<ORDER>(c.t, h);
  const int a = c.t.fv[h], b = c.t.fv[hn];
  const int t = c.a.twin[h];
  const int r = he_face<ORDER>(c.t, h);
  const f3 pab = add3(ld3(c.P, a), ld3(c.P, b));
  f3 ep;
  const double sj = c.creases ? c.a.sig[e] : 0.0;
  if (t < 0) {
    ep = mul3(0.5f, pab);
  } else {
    const int s = he_face<ORDER>(c.t, t);
    ep = mul3(0.25f, add3(pab, add3(ld3(c.P1, V + r), ld3(c.P1, V + s))));
    if (sj >= 1.0) ep = mul3(0.5f, pab);
    else if (sj > 0.0) {
      const float fs = (float)sj;
      ep = fma3(1.0f - fs, ep, mul3(fs * 0.5f, pab));
    }
  }
  st3(c.P1, V + F + e, ep);
  if (!c.sig1) return;
  const int base = edge_base(c, e);
  const int nchild = t < 0 ? 3 : 4;
  {
    double s_lo = 0.0, s_hi = 0.0;
    if (sj > 0.0) {
      const int lo = a < b ? a : b, hi = a < b ? b : a;
      const int4 cl = c.a.vcr[lo], ch = c.a.vcr[hi];
      const double si = cl.x == 2 ? c.a.sig[cl.y == e ? cl.z : cl.y] : sj;
      const double sk = ch.x == 2 ? c.a.sig[ch.y == e ? ch.z : ch.y] : sj;
      s_lo = chaikin(si, sj);
      s_hi = chaikin(sk, sj);
    }
    c.sig1[base + 0] = s_lo;
    c.sig1[base + 1] = s_hi;
    for (int i = 2; i < nchild; ++i) c.sig1[base + i] = 0.0;
  }
}

template <int ORDER>
static void cc_launch_t(int which, const CCStep &c, hipStream_t s) {
  if (which == CC_FACE)
    hipLaunchKernelGGL(k_cc_face<ORDER>, dim3(grid_for(c.t.F)), dim3(kBlock), 0, s, c);
  else if (which == CC_VERTEX)
    hipLaunchKernelGGL(k_cc_vertex<ORDER>, dim3(grid_for(c.t.V)), dim3(kBlock), 0, s, c);
  else
    hipLaunchKernelGGL(k_cc_edge<ORDER>, dim3(grid_for(c.a.E)), dim3(kBlock), 0, s, c);
}

hipError_t cc_launch(int which, const CCStep &c, hipStream_t s) {
  if (c.t.order == 4) cc_launch_t<4>(which, c, s);
  else if (c.t.order == 3) cc_launch_t<3>(which, c, s);
  else cc_launch_t<0>(which, c, s);
  return hipGetLastError();
}

}  // namespace subdiv
