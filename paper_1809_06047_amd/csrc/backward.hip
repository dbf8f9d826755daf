// Adjoint of one Catmull-Clark level on gfx950.
//
// One refinement step is linear in the vertex data, P_{k+1} = R_k P_k
// (Sec. 3.6, single-SpMV evaluation), with R_k fixed by the topology and the
// creases only. The adjoint g_k = R_k^T g_{k+1} is computed as deterministic
// transposed gathers over the same adjacency the forward step used (no
// atomics, no explicit R_k):
//
// Forward rules written as coefficients (Sec. 3.1 and 3.3, eq::CC_boundary):
//   vertex w:  S_w = a_w p_w + b_w (sum_nbrs p_j + sum_faces f_q) + d_w (p_c1 + p_c2)
//     boundary:          a = 3/4, b = 0, d = 1/8     (c1, c2 = boundary neighbours)
//     interior, smooth:  a = 1 - 2/n, b = 1/n^2, d = 0
//     interior, k >= 2 creases with blend l = min(mean sharpness, 1):
//                        a = (1-l)(1-2/n) + l (3/4 if k = 2 else 1), b = (1-l)/n^2,
//                        d = l/8 if k = 2 (c1, c2 = the crease neighbours) else 0
//   edge e = (a, b) with faces r, s:  E_e = m_e (p_a + p_b) + u_e (f_r + f_s)
//     boundary: m = 1/2, u = 0; interior with l_e = min(sigma_e, 1): m = (1-l)/4 + l/2, u = (1-l)/4
//   face q:   f_q = (1/c_q) sum_corners p
// Transposed:
//   gf_q  = ( gF_q + sum_{interior edges e of q} u_e gE_e + sum_{corners w of q} b_w gV_w ) / c_q
//   g_u   = a_u gV_u + sum_{nbrs w} b_w gV_w + sum_{faces q of u} gf_q + sum_{edges e=(u,w)} m_e gE_e
//           + sum_{w: u is c1 or c2 of w} d_w gV_w
// where u is c1/c2 of w iff the edge (u, w) is a boundary edge, or a crease
// edge with w interior and k_w = 2.
#include "subdiv_internal.h"

namespace subdiv {

struct BwdCoef {
  float a, b, d;
  int flags;  // bit 0: boundary vertex
};

// forward vertex-rule coefficients of every level-k vertex (ring walk)
template <int ORDER>
__global__ void __launch_bounds__(kBlock) k_bw_coef(BwdStep c) {
  const int v = blockIdx.x * blockDim.x + threadIdx.x;
  if (v >= c.t.V) return;
  const int h0 = c.a.vhe[v];
  const bool bnd = c.a.twin[h0] < 0;
  BwdCoef co;
  if (bnd) {
    co = BwdCoef{0.75f, 0.0f, 0.125f, 1};
  } else {
    int n = 0, k = 0;
    double ssum = 0.0;
    int h = h0;
    while (true) {
      ++n;
      if (c.a.sig) {
        const double s = c.a.sig[c.a.eid[h]];
        if (s > 0.0) {
          ++k;
          ssum += s;
        }
      }
      const int t = c.a.twin[he_prev<ORDER>(c.t, h)];
      if (t < 0 || t == h0 || n >= SUBDIV_MAX_VALENCE) break;
      h = t;
    }
    const float fn = (float)n;
    const float sa = 1.0f - 2.0f / fn, sb = 1.0f / (fn * fn);
    if (k >= 2) {
      const double s = ssum / (double)k;
      const float l = s >= 1.0 ? 1.0f : (float)s;
      co = BwdCoef{(1.0f - l) * sa + l * (k == 2 ? 0.75f : 1.0f), (1.0f - l) * sb, k == 2 ? l * 0.125f : 0.0f, 0};
    } else {
      co = BwdCoef{sa, sb, 0.0f, 0};
    }
  }
  reinterpret_cast<float4 *>(c.coef)[v] = make_float4(co.a, co.b, co.d, __int_as_float(co.flags));
}

__device__ __forceinline__ void edge_coef(const BwdStep &c, int h, float &m, float &u) {
  if (c.a.twin[h] < 0) {
    m = 0.5f;
    u = 0.0f;
    return;
  }
  const double s = c.a.sig ? c.a.sig[c.a.eid[h]] : 0.0;
  const float l = s >= 1.0 ? 1.0f : (s > 0.0 ? (float)s : 0.0f);
  m = (1.0f - l) * 0.25f + l * 0.5f;
  u = (1.0f - l) * 0.25f;
}

// adjoint of the face points, divided by the face order
template <int ORDER>
__global__ void __launch_bounds__(kBlock) k_bw_face(BwdStep c) {
  const int r = blockIdx.x * blockDim.x + threadIdx.x;
  if (r >= c.t.F) return;
  const int V = c.t.V, F = c.t.F;
  const int b = face_begin<ORDER>(c.t, r), en = face_end<ORDER>(c.t, r);
  f3 g = ld3(c.g1, V + r);
  const float4 *coef = reinterpret_cast<const float4 *>(c.coef);
  for (int h = b; h < en; ++h) {
    float m, u;
    edge_coef(c, h, m, u);
    if (u != 0.0f) g = fma3(u, ld3(c.g1, V + F + c.a.eid[h]), g);
    const int w = c.t.fv[h];
    const float bw = coef[w].y;
    if (bw != 0.0f) g = fma3(bw, ld3(c.g1, w), g);
  }
  st3(c.gf, r, mul3(1.0f / (float)(en - b), g));
}

// adjoint of the whole level at every vertex
template <int ORDER>
__global__ void __launch_bounds__(kBlock) k_bw_vertex(BwdStep c) {
  const int v = blockIdx.x * blockDim.x + threadIdx.x;
  if (v >= c.t.V) return;
  const int V = c.t.V, F = c.t.F;
  const float4 *coef = reinterpret_cast<const float4 *>(c.coef);
  const float4 cv = coef[v];
  f3 g = mul3(cv.x, ld3(c.g1, v));
  const int h0 = c.a.vhe[v];
  int h = h0, n = 0;
  while (true) {
    const int w = c.t.fv[he_next<ORDER>(c.t, h)];
    const float4 cw = coef[w];
    const f3 gw = ld3(c.g1, w);
    float m, u;
    edge_coef(c, h, m, u);
    g = fma3(cw.y, gw, g);                                   // v is a neighbour in w's smooth rule
    g = fma3(m, ld3(c.g1, V + F + c.a.eid[h]), g);          // edge point of (v, w)
    g = add3(g, ld3(c.gf, he_face<ORDER>(c.t, h)));         // face point of the face of h
    const bool bedge = c.a.twin[h] < 0;
    const bool cedge = c.a.sig && c.a.sig[c.a.eid[h]] > 0.0 && !(__float_as_int(cw.w) & 1);
    if (bedge || cedge) g = fma3(cw.z, gw, g);               // v is c1/c2 of w
    ++n;
    const int hp = he_prev<ORDER>(c.t, h);
    const int t = c.a.twin[hp];
    if (t < 0) {
      // last edge (u -> v) of a boundary fan: neighbour u, a boundary edge
      const int uu = c.t.fv[hp];
      const float4 cu = coef[uu];
      const f3 gu = ld3(c.g1, uu);
      g = fma3(cu.y, gu, g);
      g = fma3(0.5f, ld3(c.g1, V + F + c.a.eid[hp]), g);
      g = fma3(cu.z, gu, g);
      break;
    }
    if (t == h0 || n >= SUBDIV_MAX_VALENCE) break;
    h = t;
  }
  st3(c.g0, v, g);
}

hipError_t bw_launch(int which, const BwdStep &c, hipStream_t s) {
  const unsigned gv = grid_for(c.t.V), gf = grid_for(c.t.F);
#define SUBDIV_BW(ORD)                                                                  \
  do {                                                                                  \
    if (which == BW_COEF) hipLaunchKernelGGL(k_bw_coef<ORD>, dim3(gv), dim3(kBlock), 0, s, c);   \
    else if (which == BW_FACE) hipLaunchKernelGGL(k_bw_face<ORD>, dim3(gf), dim3(kBlock), 0, s, c); \
    else hipLaunchKernelGGL(k_bw_vertex<ORD>, dim3(gv), dim3(kBlock), 0, s, c);                 \
  } while (0)
  if (c.t.order == 4) SUBDIV_BW(4);
  else if (c.t.order == 3) SUBDIV_BW(3);
  else SUBDIV_BW(0);
#undef SUBDIV_BW
  return hipGetLastError();
}

}  // namespace subdiv
