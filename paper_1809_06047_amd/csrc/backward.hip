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

__device__ __forceinline__ BwdCoef smooth_or_blend(int n, int k, double ssum) {
  const float fn = (float)n;
  const float sa = 1.0f - 2.0f / fn, sb = 1.0f / (fn * fn);
  if (k >= 2) {
    const double s = ssum / (double)k;
    const float l = s >= 1.0 ? 1.0f : (float)s;
    return BwdCoef{(1.0f - l) * sa + l * (k == 2 ? 0.75f : 1.0f), (1.0f - l) * sb, k == 2 ? l * 0.125f : 0.0f, 0};
  }
  return BwdCoef{sa, sb, 0.0f, 0};
}

// forward vertex-rule coefficients of every level-k vertex. On a level
// refined from quads, the face points of level k-1 are interior, of valence
// 4 and on no crease; an edge point EP(e) has valence 4 unless e is a
// boundary edge, and its only possible creases are the two halves of e, the
// level-k edges base(e) and base(e) + 1 (base(e) = 4 e - boundary edges
// before e). Only the older vertices walk their ring.
template <int BLK, int ORDER>
__global__ void __launch_bounds__(BLK) k_bw_coef(BwdStep c) {
  const int v = blockIdx.x * blockDim.x + threadIdx.x;
  if (v >= c.t.V) return;
  float4 *out = reinterpret_cast<float4 *>(c.coef);
  if (c.Vp > 0 && v >= c.Vp) {
    BwdCoef co{0.5f, 0.0625f, 0.0f, 0};  // valence 4, smooth
    if (v >= c.Vp + c.Fp) {
      if (c.a.twin[c.a.vhe[v]] < 0) {
        co = BwdCoef{0.75f, 0.0f, 0.125f, 1};
      } else if (c.a.sig) {
        const int e = v - c.Vp - c.Fp;
        const int base = 4 * e - (c.bscan_p ? c.bscan_p[e] : 0);
        const double s0 = c.a.sig[base], s1 = c.a.sig[base + 1];
        const int k = (s0 > 0.0) + (s1 > 0.0);
        if (k == 2) co = smooth_or_blend(4, 2, s0 + s1);
      }
    }
    out[v] = make_float4(co.a, co.b, co.d, __int_as_float(co.flags));
    return;
  }
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
    co = smooth_or_blend(n, k, ssum);
  }
  out[v] = make_float4(co.a, co.b, co.d, __int_as_float(co.flags));
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

// Per face: the adjoint of its face point, divided by the face order, and
// then every half-edge's share of its origin's gather. Half-edge h (u -> w)
// carries the terms of g_u that come with the edge (u, w) and the face of h:
//   term(h) = b_w gV_w + m_e gE_e + gf_q (+ d_w gV_w when u is c1/c2 of w),
// so the vertex kernel adds one 12-byte term per ring step instead of
// gathering six arrays at every step.
template <int BLK, int ORDER>
__global__ void __launch_bounds__(BLK) k_bw_face(BwdStep c) {
  const int rid = blockIdx.x * blockDim.x + threadIdx.x;
  const int V = c.t.V, F = c.t.F;
  const float4 *coef = reinterpret_cast<const float4 *>(c.coef);
  if (F <= 0) return;
  if constexpr (ORDER > 0) {
    // uniform faces: the corners and edges are loaded once, and the terms of
    // the wave's faces (contiguous) leave through LDS as whole lines
    __shared__ uint32_t stage[BLK / 64][64 * (3 * ORDER | 1)];
    const bool valid = rid < F;
    const int r = valid ? rid : F - 1;
    const int l = threadIdx.x & 63;
    const long long rw = (long long)rid - l;  // first face of the wave
    const int cnt = (int)min(64ll, (long long)F - rw) * 3 * ORDER;
    int w[ORDER];
    float4 cw[ORDER];
    f3 gw[ORDER], ge[ORDER];
    float m[ORDER], u[ORDER];
    f3 g = ld3(c.g1, V + r);
#pragma unroll
    for (int i = 0; i < ORDER; ++i) {
      const int h = ORDER * r + i;
      w[i] = c.t.fv[h];
      cw[i] = coef[w[i]];
      gw[i] = ld3(c.g1, w[i]);
      ge[i] = ld3(c.g1, V + F + c.a.eid[h]);
      edge_coef(c, h, m[i], u[i]);
    }
#pragma unroll
    for (int i = 0; i < ORDER; ++i) {
      if (u[i] != 0.0f) g = fma3(u[i], ge[i], g);
      if (cw[i].y != 0.0f) g = fma3(cw[i].y, gw[i], g);
    }
    const f3 gq = mul3(1.0f / (float)ORDER, g);
    uint32_t out[3 * ORDER];
#pragma unroll
    for (int i = 0; i < ORDER; ++i) {
      const int h = ORDER * r + i, n = (i + 1) % ORDER;  // h runs from w[i] to w[n]
      f3 t = add3(fma3(cw[n].y, gw[n], mul3(m[i], ge[i])), gq);
      const bool bedge = c.a.twin[h] < 0;
      const bool cedge = c.a.sig && c.a.sig[c.a.eid[h]] > 0.0 && !(__float_as_int(cw[n].w) & 1);
      if (bedge || cedge) t = fma3(cw[n].z, gw[n], t);  // w[i] is c1/c2 of w[n]
      out[3 * i + 0] = __float_as_uint(t.x);
      out[3 * i + 1] = __float_as_uint(t.y);
      out[3 * i + 2] = __float_as_uint(t.z);
    }
    wave_store<3 * ORDER>(stage[threadIdx.x >> 6], out, reinterpret_cast<uint32_t *>(c.term) + 3 * ORDER * rw, l,
                          cnt);
  } else {
    if (rid >= F) return;
    const int r = rid;
    const int b = face_begin<ORDER>(c.t, r), en = face_end<ORDER>(c.t, r);
    f3 g = ld3(c.g1, V + r);
    for (int h = b; h < en; ++h) {
      float m, u;
      edge_coef(c, h, m, u);
      if (u != 0.0f) g = fma3(u, ld3(c.g1, V + F + c.a.eid[h]), g);
      const float bw = coef[c.t.fv[h]].y;
      if (bw != 0.0f) g = fma3(bw, ld3(c.g1, c.t.fv[h]), g);
    }
    const f3 gq = mul3(1.0f / (float)(en - b), g);
    for (int h = b; h < en; ++h) {
      const int w = c.t.fv[he_next<ORDER>(c.t, h)];
      const float4 cw = coef[w];
      const f3 gw = ld3(c.g1, w);
      float m, u;
      edge_coef(c, h, m, u);
      f3 t = add3(fma3(cw.y, gw, mul3(m, ld3(c.g1, V + F + c.a.eid[h]))), gq);
      const bool bedge = c.a.twin[h] < 0;
      const bool cedge = c.a.sig && c.a.sig[c.a.eid[h]] > 0.0 && !(__float_as_int(cw.w) & 1);
      if (bedge || cedge) t = fma3(cw.z, gw, t);  // u is c1/c2 of w
      st3(c.term, h, t);
    }
  }
}

// adjoint of the whole level at every vertex: its own vertex rule plus the
// terms of its outgoing half-edges, and on a boundary the incoming boundary
// edge (u -> v), whose half-edge belongs to u
template <int BLK, int ORDER>
__global__ void __launch_bounds__(BLK) k_bw_vertex(BwdStep c) {
  const int v = blockIdx.x * blockDim.x + threadIdx.x;
  if (v >= c.t.V) return;
  const int V = c.t.V, F = c.t.F;
  const float4 *coef = reinterpret_cast<const float4 *>(c.coef);
  f3 g = mul3(coef[v].x, ld3(c.g1, v));
  if (c.Vp > 0 && v >= c.Vp && v < c.Vp + c.Fp) {
    // face point of level-k-1 face p: its half-edges are slot 2 of p's four
    // children, in ring order from its canonical start (child 0)
    const float *tp = c.term + 48ll * (v - c.Vp);
#pragma unroll
    for (int i = 0; i < 4; ++i) g = add3(g, ld3(tp, 4 * i + 2));
    st3(c.g0, v, g);
    return;
  }
  const int h0 = c.a.vhe[v];
  if (ORDER == 4 && c.Vp > 0 && v >= c.Vp + c.Fp) {
    // edge point of parent edge e' (interior): its four half-edges in closed
    // form, in the walk's order from the canonical start: with a the half-edge
    // of e' whose child carries the start, the twin of child a's slot 0 is
    // slot 3 of child bn = next(b) across, b the other half-edge of e', and
    // the ring is 4a+1, 4bn+3, 4b+1, 4an+3 (an = next(a)), from its first or
    // its last entry
    const int a0 = (h0 & 3) == 1 ? (h0 >> 2) : (((h0 >> 2) & ~3) | (((h0 >> 2) + 3) & 3));
    const int tw = c.a.twin[4 * a0];
    if (tw >= 0) {
      const int bn = tw >> 2, b0 = (bn & ~3) | ((bn + 3) & 3), an = (a0 & ~3) | ((a0 + 1) & 3);
      const int cyc[4] = {4 * a0 + 1, 4 * bn + 3, 4 * b0 + 1, 4 * an + 3};
      const bool at0 = (h0 & 3) == 1;
      f3 tv[4];
#pragma unroll
      for (int j = 0; j < 4; ++j) tv[j] = ld3(c.term, at0 ? cyc[j] : cyc[(j + 3) & 3]);
#pragma unroll
      for (int j = 0; j < 4; ++j) g = add3(g, tv[j]);
      st3(c.g0, v, g);
      return;
    }
  }
  // neighbour u of the last, boundary edge (incoming half-edge hp): v is in
  // u's smooth rule (b_u), takes half of the edge point, and is one of u's two
  // boundary neighbours
  auto boundary_terms = [&](int hp) {
    const int uu = c.t.fv[hp];
    const float4 cu = coef[uu];
    const f3 gu = ld3(c.g1, uu);
    g = fma3(cu.y, gu, g);
    g = fma3(0.5f, ld3(c.g1, V + F + c.a.eid[hp]), g);
    g = fma3(cu.z, gu, g);
  };
  // the fan first (only the twin loads in sequence), then every term at once,
  // added in the same order; longer fans walk one step at a time
  constexpr int kFan = 8;
  int hs[kFan], n = 0, h = h0, hb = -1;
  bool go = true;
#pragma unroll
  for (int i = 0; i < kFan; ++i) {
    hs[i] = h;  // past the end: repeats the last half-edge (loads stay in bounds)
    if (go) {
      n = i + 1;
      const int hp = he_prev<ORDER>(c.t, h);
      const int t = c.a.twin[hp];
      if (t < 0) {
        hb = hp;
        go = false;
      } else if (t == h0) {
        go = false;
      } else {
        h = t;
      }
    }
  }
  if (!go) {
    f3 tv[kFan];
#pragma unroll
    for (int i = 0; i < kFan; ++i) tv[i] = ld3(c.term, hs[i]);
#pragma unroll
    for (int i = 0; i < kFan; ++i)
      if (i < n) g = add3(g, tv[i]);
    if (hb >= 0) boundary_terms(hb);
    st3(c.g0, v, g);
    return;
  }
  h = h0;
  n = 0;
  while (true) {
    g = add3(g, ld3(c.term, h));
    ++n;
    const int hp = he_prev<ORDER>(c.t, h);
    const int t = c.a.twin[hp];
    if (t < 0) {
      boundary_terms(hp);
      break;
    }
    if (t == h0 || n >= SUBDIV_MAX_VALENCE) break;
    h = t;
  }
  st3(c.g0, v, g);
}

hipError_t bw_launch(int which, const BwdStep &c, hipStream_t s) {
#define SUBDIV_BW(ORD)                                                           \
  do {                                                                           \
    if (which == BW_COEF) SUBDIV_LAUNCH_TUNED_T(TK_BW_COEF, c.t.V, s, k_bw_coef, ORD, c);  \
    else if (which == BW_FACE) SUBDIV_LAUNCH_TUNED_T(TK_BW_FACE, c.t.F, s, k_bw_face, ORD, c); \
    else SUBDIV_LAUNCH_TUNED_T(TK_BW_VERTEX, c.t.V, s, k_bw_vertex, ORD, c);               \
  } while (0)
  if (c.t.order == 4) SUBDIV_BW(4);
  else if (c.t.order == 3) SUBDIV_BW(3);
  else SUBDIV_BW(0);
#undef SUBDIV_BW
  return hipGetLastError();
}

}  // namespace subdiv
