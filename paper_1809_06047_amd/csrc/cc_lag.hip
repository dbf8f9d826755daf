// Catmull-Clark levels k >= 1 on gfx950, computed from the adjacency of the
// parent level m = k-1 (the level k was refined from).
//
// Level k is itself the Catmull-Clark refinement of level m, so everything
// the build step of level k would produce (its mesh matrix M_k, the mapped
// products E_k, F_k) is a closed-form function of M_m and of E_m, F_m
// (Sec. 3.2 "Topology refinement"):
//   * face q of level k is child j of parent face p (q = col_ptr_m[p] + j =
//     parent half-edge h) with corners (v_j, EP(e_j), FP(p), EP(e_{j-1})),
//     EP(e) = |v_m| + |f_m| + e, FP(p) = |v_m| + p;
//   * every level-k edge has an edge point EP(e) as its higher end, so the
//     upper triangle of E_k enumerates the children of parent edge e at
//     base(e) + rank, base(e) = 4 e - (boundary edges before e), rank over
//     the ascending lower neighbours lo(e), hi(e), FP(min face), FP(max face);
//   * F_k (twin half-edges) follows from F_m.
// The kernels therefore iterate over the parent level's faces, edges and
// vertices, whose arrays are 4x smaller than level k's, and read every
// level-k quantity in the order it is laid out:
//   k_lag_group  (per parent face p) : face points of p's children (eq:spla_fp),
//                                      the vertex point of FP(p), child topology
//                                      of level k+1, level-k rows of M, E, F
//   k_lag_vertex (per parent vertex) : vertex points of the level-m vertices
//                                      (ring walk on level m), crease valency
//   k_lag_edge   (per parent edge e) : the 3-4 edge points of e's children, the
//                                      vertex point of EP(e), crease inheritance
//                                      (Chaikin rule), edge -> half-edge map
// The rules are those of Sec. 3.1 / 3.3 (see cc.hip). Sums over a symmetric
// pair are written as balanced trees of commutative additions, so results do
// not depend on which half-edge of an edge is its owner.
#include "subdiv_internal.h"

namespace subdiv {

__device__ __forceinline__ double chaikin_lag(double si, double sj) {
#pragma clang fp contract(off)
  const double t = 0.25 * (si + 3.0 * sj) - 1.0;  // this operation order, no fused multiply-add
  return t > 0.0 ? t : 0.0;
}

__device__ __forceinline__ int lag_base(const LagStep &c, int e) { return 4 * e - (c.bnd ? c.am.bscan[e] : 0); }

template <int OM>
__device__ __forceinline__ int face_of(const LagStep &c, int h) {
  return he_face<OM>(c.tm, h);
}

// ------------------------------------------------------------- group kernel
template <int BLK, int OM>
__global__ void __launch_bounds__(BLK) k_lag_group(LagStep c) {
  const int p = blockIdx.x * blockDim.x + threadIdx.x;
  if (p >= c.tm.F) return;
  const Topo &tm = c.tm;
  const int Vm = tm.V, VFm = tm.V + tm.F;
  const int Vk = c.Vk, VFk = c.Vk + c.Fk;
  const int b = face_begin<OM>(tm, p), en = face_end<OM>(tm, p), n = en - b;
  const int FP = Vm + p;
  const f3 pFP = ld3(c.Pk, FP);
  f3 sum_ep{0.f, 0.f, 0.f}, sum_f{0.f, 0.f, 0.f};
  const bool emit = c.ak.twin != nullptr;
  // previous corner (slot n-1) for child 0
  int hp = en - 1;
  int vprev = tm.fv[hp], eprev = c.am.eid[hp], tprev = c.am.twin[hp];
  f3 pEPprev = ld3(c.Pk, VFm + eprev);
  for (int h = b; h < en; ++h) {
    const int hn = (h + 1 == en) ? b : h + 1;
    const int v = tm.fv[h], e = c.am.eid[h], t = c.am.twin[h];
    const int vnext = tm.fv[hn];
    const f3 pv = ld3(c.Pk, v), pEP = ld3(c.Pk, VFm + e);
    // face point of level-k face q = h: corners (v, EP(e), FP, EP(eprev))
    const f3 f = mul3(0.25f, add3(add3(pv, pEP), add3(pFP, pEPprev)));
    st3(c.P1, Vk + h, f);
    sum_ep = add3(sum_ep, pEP);
    sum_f = add3(sum_f, f);
    // level-k edge ids of the 4 half-edges of q (upper triangle of E_k)
    const int bj = lag_base(c, e), bp = lag_base(c, eprev);
    const int s = t < 0 ? -1 : face_of<OM>(c, t), sp = tprev < 0 ? -1 : face_of<OM>(c, tprev);
    const int k0 = bj + (v > vnext);
    const int k1 = bj + 2 + (s >= 0 && s < p);
    const int k2 = bp + 2 + (sp >= 0 && sp < p);
    const int k3 = bp + (v > vprev);
    const int c0 = v, c1 = VFm + e, c2 = FP, c3 = VFm + eprev;
    if (c.fvk) reinterpret_cast<int4 *>(c.fvk)[h] = make_int4(c0, c1, c2, c3);
    if (emit) {
      const int tn = t < 0 ? -1 : he_next<OM>(tm, t);
      reinterpret_cast<int4 *>(c.ak.twin)[h] =
          make_int4(t < 0 ? -1 : 4 * tn + 3, 4 * hn + 2, 4 * hp + 1, tprev < 0 ? -1 : 4 * tprev);
      reinterpret_cast<int4 *>(c.ak.eid)[h] = make_int4(k0, k1, k2, k3);
    }
    if (c.fv1) {
      // children of q at level k+1: (corner_i, EP_k(k_i), FP_k(q), EP_k(k_{i-1}))
      int4 *o = reinterpret_cast<int4 *>(c.fv1) + 4ll * h;
      const int fq = Vk + h;
      o[0] = make_int4(c0, VFk + k0, fq, VFk + k3);
      o[1] = make_int4(c1, VFk + k1, fq, VFk + k0);
      o[2] = make_int4(c2, VFk + k2, fq, VFk + k1);
      o[3] = make_int4(c3, VFk + k3, fq, VFk + k2);
    }
    hp = h;
    vprev = v;
    eprev = e;
    tprev = t;
    pEPprev = pEP;
  }
  // vertex point of FP(p): interior, valence n, neighbours EP(e_j), faces = children
  const float fn = (float)n;
  st3(c.P1, FP, fma3(1.0f - 2.0f / fn, pFP, mul3(1.0f / (fn * fn), add3(sum_ep, sum_f))));
  if (emit) c.ak.vhe[FP] = 4 * b + 2;
}

// ------------------------------------------------------------ vertex kernel
template <int BLK, int OM>
__global__ void __launch_bounds__(BLK) k_lag_vertex(LagStep c) {
  const int v = blockIdx.x * blockDim.x + threadIdx.x;
  if (v >= c.tm.V) return;
  const Topo &tm = c.tm;
  const int VFm = tm.V + tm.F, Vk = c.Vk;
  const int h0 = c.am.vhe[v];
  const f3 p = ld3(c.Pk, v);
  const bool creases = c.sigk != nullptr;
  f3 sum_ep{0.f, 0.f, 0.f}, sum_f{0.f, 0.f, 0.f};
  int n = 0, k = 0, cv0 = -1, cv1 = -1, ce0 = -1, ce1 = -1, ep_last = -1;
  double ssum = 0.0;
  int h = h0;
  while (true) {
    const int e = c.am.eid[h];
    const int EP = VFm + e;
    sum_ep = add3(sum_ep, ld3(c.Pk, EP));
    sum_f = add3(sum_f, ld3(c.P1, Vk + h));  // face point of level-k face h (v at slot 0)
    ++n;
    if (creases) {
      const int w = tm.fv[he_next<OM>(tm, h)];
      const int eps = lag_base(c, e) + (v > w);  // level-k edge (v, EP)
      const double s = c.sigk[eps];
      if (s > 0.0) {
        if (k == 0) { cv0 = EP; ce0 = eps; } else if (k == 1) { cv1 = EP; ce1 = eps; }
        ++k;
        ssum += s;
      }
    }
    const int hpv = he_prev<OM>(tm, h);
    const int t = c.am.twin[hpv];
    if (t < 0) {  // boundary: the incoming boundary half-edge u -> v ends the fan
      const int e2 = c.am.eid[hpv];
      ep_last = VFm + e2;
      if (creases) {
        const int u = tm.fv[hpv];
        const int eps = lag_base(c, e2) + (v > u);
        const double s = c.sigk[eps];
        if (s > 0.0) {
          if (k == 0) { cv0 = ep_last; ce0 = eps; } else if (k == 1) { cv1 = ep_last; ce1 = eps; }
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
  if (ep_last >= 0) {  // boundary vertex: 3/4 p + 1/8 (two boundary neighbours at level k)
    const int ep_first = VFm + c.am.eid[h0];
    S = fma3(0.75f, p, mul3(0.125f, add3(ld3(c.Pk, ep_first), ld3(c.Pk, ep_last))));
  } else {
    const float fn = (float)n;
    S = fma3(1.0f - 2.0f / fn, p, mul3(1.0f / (fn * fn), add3(sum_ep, sum_f)));
    if (creases && k >= 2) {
      const f3 sharp = (k == 2) ? fma3(0.75f, p, mul3(0.125f, add3(ld3(c.Pk, cv0), ld3(c.Pk, cv1)))) : p;
      const double s = ssum / (double)k;
      if (s >= 1.0) S = sharp;
      else {
        const float fs = (float)s;
        S = fma3(1.0f - fs, S, mul3(fs, sharp));
      }
    }
  }
  st3(c.P1, v, S);
  if (creases && c.vcrk) c.vcrk[v] = make_int4(k, ce0, ce1, 0);
  if (c.ak.vhe) c.ak.vhe[v] = 4 * h0;
}

// -------------------------------------------------------------- edge kernel
template <int BLK, int OM>
__global__ void __launch_bounds__(BLK) k_lag_edge(LagStep c) {
  const int eid = blockIdx.x * blockDim.x + threadIdx.x;
  const bool valid = eid < c.am.E;
  const int e = valid ? eid : c.am.E - 1;  // every lane takes part in the staged store
  const Topo &tm = c.tm;
  const int Vm = tm.V, VFm = tm.V + tm.F;
  const int Vk = c.Vk, VFk = c.Vk + c.Fk;
  const int h = c.am.e2h[e];
  const int t = c.am.twin[h];
  const int hn = he_next<OM>(tm, h);
  const int a = tm.fv[h], bv = tm.fv[hn];
  const int pf = face_of<OM>(c, h);
  const int EP = VFm + e;
  const int base = lag_base(c, e);
  const f3 pa = ld3(c.Pk, a), pb = ld3(c.Pk, bv), pEP = ld3(c.Pk, EP), pFPp = ld3(c.Pk, Vm + pf);
  const f3 fh = ld3(c.P1, Vk + h), fhn = ld3(c.P1, Vk + hn);
  const bool creases = c.sigk != nullptr;
  const int ra = a < bv ? 0 : 1;  // rank of (a, EP) among e's children
  const double sa = creases ? c.sigk[base + ra] : 0.0, sb = creases ? c.sigk[base + 1 - ra] : 0.0;
  f3 ea, eb, S, ec[4];
  int s = -1, tn = -1;
  if (t < 0) {
    ea = mul3(0.5f, add3(pa, pEP));
    eb = mul3(0.5f, add3(pb, pEP));
    // boundary edge point vertex: 3/4 p + 1/8 (a + b)
    S = fma3(0.75f, pEP, mul3(0.125f, add3(pa, pb)));
    ec[2] = mul3(0.25f, add3(add3(pFPp, pEP), add3(fh, fhn)));
  } else {
    s = face_of<OM>(c, t);
    tn = he_next<OM>(tm, t);
    const f3 pFPs = ld3(c.Pk, Vm + s);
    const f3 ft = ld3(c.P1, Vk + t), ftn = ld3(c.P1, Vk + tn);
    ea = mul3(0.25f, add3(add3(pa, pEP), add3(fh, ftn)));
    eb = mul3(0.25f, add3(add3(pb, pEP), add3(fhn, ft)));
    const f3 ep_p = mul3(0.25f, add3(add3(pFPp, pEP), add3(fh, fhn)));
    const f3 ep_s = mul3(0.25f, add3(add3(pFPs, pEP), add3(ft, ftn)));
    ec[pf < s ? 2 : 3] = ep_p;
    ec[pf < s ? 3 : 2] = ep_s;
    // interior edge point vertex: valence 4, neighbours a, b, FP(p), FP(s)
    const f3 nb = add3(add3(pa, pb), add3(pFPp, pFPs));
    const f3 fs = add3(add3(fh, fhn), add3(ft, ftn));
    S = fma3(0.5f, pEP, mul3(1.0f / 16.0f, add3(nb, fs)));
    if (creases) {
      const int kk = (sa > 0.0) + (sb > 0.0);
      if (kk == 2) {
        const f3 sharp = fma3(0.75f, pEP, mul3(0.125f, add3(pa, pb)));
        const double sv = (sa + sb) * 0.5;
        if (sv >= 1.0) S = sharp;
        else {
          const float fsv = (float)sv;
          S = fma3(1.0f - fsv, S, mul3(fsv, sharp));
        }
      }
    }
    // crease edges among the halves (boundary halves stay midpoints)
    if (sa >= 1.0) ea = mul3(0.5f, add3(pa, pEP));
    else if (sa > 0.0) {
      const float w = (float)sa;
      ea = fma3(1.0f - w, ea, mul3(w * 0.5f, add3(pa, pEP)));
    }
    if (sb >= 1.0) eb = mul3(0.5f, add3(pb, pEP));
    else if (sb > 0.0) {
      const float w = (float)sb;
      eb = fma3(1.0f - w, eb, mul3(w * 0.5f, add3(pb, pEP)));
    }
  }
  ec[ra] = ea;
  ec[1 - ra] = eb;
  const int nchild = t < 0 ? 3 : 4;
  {
    // the children's edge points, VFk + base .. base + nchild - 1, are one
    // contiguous run over the wave (base(e + 1) = base(e) + nchild(e)): they
    // leave through LDS as runs of 64 consecutive dwords
    __shared__ uint32_t stage[BLK / 64][64 * 12];
    const int w = threadIdx.x >> 6, l = threadIdx.x & 63;
    uint32_t *lds = stage[w];
    const int base0 = __shfl(base, 0, 64);
    const int end = __shfl(base + nchild, min(63, c.am.E - 1 - (eid - l)), 64);
    const int off = 3 * (base - base0);
#pragma unroll
    for (int r = 0; r < 4; ++r)
      if (r < nchild) {
        lds[off + 3 * r + 0] = __float_as_uint(ec[r].x);
        lds[off + 3 * r + 1] = __float_as_uint(ec[r].y);
        lds[off + 3 * r + 2] = __float_as_uint(ec[r].z);
      }
    __builtin_amdgcn_wave_barrier();
    const int count = (eid - l < c.am.E) ? 3 * (end - base0) : 0;
    uint32_t *dst = reinterpret_cast<uint32_t *>(c.P1 + 3ll * (VFk + base0));
    run_store(lds, dst, count, l);
  }
  if (!valid) return;
  st3(c.P1, EP, S);
  if (c.edges_k) {  // (lo, hi) of level-k edges, in id order
    int2 *o = reinterpret_cast<int2 *>(c.edges_k);
    o[base + ra] = make_int2(a, EP);
    o[base + 1 - ra] = make_int2(bv, EP);
    if (t < 0) o[base + 2] = make_int2(Vm + pf, EP);
    else {
      o[base + 2] = make_int2(Vm + (pf < s ? pf : s), EP);
      o[base + 3] = make_int2(Vm + (pf < s ? s : pf), EP);
    }
  }
  if (c.ak.e2h) {
    const int hx0 = 4 * h, hx1 = 4 * hn + 3;
    c.ak.e2h[base + ra] = hx0;
    c.ak.e2h[base + 1 - ra] = hx1;
    if (t < 0) {
      c.ak.e2h[base + 2] = 4 * h + 1;
      c.ak.vhe[EP] = hx1;
    } else {
      c.ak.e2h[base + (pf < s ? 2 : 3)] = 4 * h + 1;
      c.ak.e2h[base + (pf < s ? 3 : 2)] = 4 * t + 1;
      const int m0 = min(4 * h + 1, 4 * hn + 3), m1 = min(4 * t + 1, 4 * tn + 3);
      c.ak.vhe[EP] = min(m0, m1);
    }
    if (c.bnd) {
      const int b2 = 2 * c.am.bscan[e];
      for (int i = 0; i < nchild; ++i) c.ak.bscan[base + i] = b2 + (t < 0 ? (i < 2 ? i : 2) : 0);
    }
  }
  if (c.sig1) {
    // children of the level-k edges of e, at level k+1: base_k(eps) + rank
    const int b2 = c.bnd ? 2 * c.am.bscan[e] : 0;
    for (int r = 0; r < nchild; ++r) {
      const int eps = base + r;
      const int bs = c.bnd ? b2 + (t < 0 ? (r < 2 ? r : 2) : 0) : 0;
      const int base1 = 4 * eps - bs;
      const int nc1 = (t < 0 && r < 2) ? 3 : 4;  // a boundary half has one face
      double c0 = 0.0, c1 = 0.0;
      if (r < 2) {
        const double sj = (r == ra) ? sa : sb;
        if (sj > 0.0) {
          const int x = (r == ra) ? a : bv;  // the old end of the half (its lower end)
          const int4 cx = c.vcrk[x];
          const double si = cx.x == 2 ? c.sigk[cx.y == eps ? cx.z : cx.y] : sj;
          const double so = (r == ra) ? sb : sa;  // the other half at EP
          const double sk = (so > 0.0) ? so : sj;
          c0 = chaikin_lag(si, sj);
          c1 = chaikin_lag(sk, sj);
        }
      }
      c.sig1[base1 + 0] = c0;
      c.sig1[base1 + 1] = c1;
      for (int i = 2; i < nc1; ++i) c.sig1[base1 + i] = 0.0;
    }
  }
}

template <int OM>
static void lag_launch_t(int which, const LagStep &c, hipStream_t s) {
  if (which == LAG_GROUP)
    SUBDIV_LAUNCH_TUNED_T(TK_LAG_GROUP, c.tm.F, s, k_lag_group, OM, c);
  else if (which == LAG_VERTEX)
    SUBDIV_LAUNCH_TUNED_T(TK_LAG_VERTEX, c.tm.V, s, k_lag_vertex, OM, c);
  else
    SUBDIV_LAUNCH_TUNED_T(TK_LAG_EDGE, c.am.E, s, k_lag_edge, OM, c);
}

hipError_t lag_launch(int which, const LagStep &c, hipStream_t s) {
  if (c.tm.order == 4) lag_launch_t<4>(which, c, s);
  else if (c.tm.order == 3) lag_launch_t<3>(which, c, s);
  else lag_launch_t<0>(which, c, s);
  return hipGetLastError();
}


// ===========================================================================
// Levels whose grandparent level g = m-1 is also all quads: the level-m
// vertices fall into three classes by the corner they occupy in a level-m
// face p = child j of grandparent quad pg (corners v_j, EP_g(e_j), FP_g(pg),
// EP_g(e_{j-1})):
//   corner 2: FP_g(pg), valence 4, its ring is corner 2 of the four siblings
//             4pg..4pg+3 (four adjacent lanes: a quad reduction);
//   corner 1: EP_g(e_j), valence 4, half of its ring is corner 1 of p and
//             corner 3 of the next sibling (lane (j+1)&3); the other half lies
//             in the quad on the far side of e_j;
//   corner 0: a vertex of level g, whose ring is walked on level g.
// Each corner's ring term (edge point of the level-k edge leaving it plus the
// face point of its level-k corner face) is formed once, by the thread that
// owns the face, in face order.
// Creases: a level-k edge can only be sharp if its parent level-m edge is a
// half of a sharp grandparent edge, so FP_g vertices are never on a crease,
// an EP_g(e) vertex has at most the two children of the halves of e (level-m
// ids base_g(e) + 0/1, their children at EP_g at base_m(.) + 1), and a level-g
// vertex v meets the children base_m(eid_m(4h)) + 0 of the level-m edges
// (v, EP_g) met on its ring walk. The crease rules are those of the general
// vertex kernel above, which these kernels replace on such levels.
// ===========================================================================

__device__ __forceinline__ f3 shfl3(f3 v, int src, int width) {
  return f3{__shfl(v.x, src, width), __shfl(v.y, src, width), __shfl(v.z, src, width)};
}
__device__ __forceinline__ f3 shfl_xor3(f3 v, int mask, int width) {
  return f3{__shfl_xor(v.x, mask, width), __shfl_xor(v.y, mask, width), __shfl_xor(v.z, mask, width)};
}

template <int BLK>
__global__ void __launch_bounds__(BLK) k_lag2_group(Lag2Step c) {
  const LagStep &L = c.s;
  const int pid = blockIdx.x * blockDim.x + threadIdx.x;
  const bool valid = pid < L.tm.F;  // F_m is a multiple of 4: quads of lanes are complete
  const int p = valid ? pid : L.tm.F - 1;
  const int j = p & 3, pg = p >> 2;
  const int Vm = L.tm.V, VFm = L.tm.V + L.tm.F;
  const int Vk = L.Vk, VFk = L.Vk + L.Fk;
  // the parent rows are read once here: non-temporal loads, so they do not
  // displace the positions gathered from L2 (the edge kernel after this one
  // reads some of them again, a smaller cost than this kernel's gain)
  auto ntl = [](const int32_t *a, int i) {
    const v4i32 x = __builtin_nontemporal_load(reinterpret_cast<const v4i32 *>(a) + i);
    return make_int4(x[0], x[1], x[2], x[3]);
  };
  const int4 q = ntl(L.tm.fv, p);
  const int4 ed = ntl(L.am.eid, p);
  const int4 tq = ntl(L.am.twin, p);
  const int cv[4] = {q.x, q.y, q.z, q.w};
  const int e[4] = {ed.x, ed.y, ed.z, ed.w};
  const int tw[4] = {tq.x, tq.y, tq.z, tq.w};
  const int FP = Vm + p;
  const f3 pFP = ld3(L.Pk, FP);
  f3 pc[4], pe[4], f[4];
#pragma unroll
  for (int i = 0; i < 4; ++i) {
    pc[i] = ld3(L.Pk, cv[i]);
    pe[i] = ld3(L.Pk, VFm + e[i]);
  }
#pragma unroll
  for (int i = 0; i < 4; ++i) f[i] = mul3(0.25f, add3(add3(pc[i], pe[i]), add3(pFP, pe[(i + 3) & 3])));
  int base[4];
#pragma unroll
  for (int i = 0; i < 4; ++i) base[i] = lag_base(L, e[i]);
  int kk[4][4];
#pragma unroll
  for (int i = 0; i < 4; ++i) {
    const int ip = (i + 3) & 3;
    const int s = tw[i] < 0 ? -1 : (tw[i] >> 2), sp = tw[ip] < 0 ? -1 : (tw[ip] >> 2);
    kk[i][0] = base[i] + (cv[i] > cv[(i + 1) & 3]);
    kk[i][1] = base[i] + 2 + (s >= 0 && s < p);
    kk[i][2] = base[ip] + 2 + (sp >= 0 && sp < p);
    kk[i][3] = base[ip] + (cv[i] > cv[ip]);
  }
  // per-face outputs are contiguous over the wave (face p owns [16 p, 16 p + 16)
  // of every level-k row array and 12 floats of face points): they leave
  // through the wave's LDS slice as whole lines
  __shared__ int4 stage[BLK / 64][32 * 17];
  const int w = threadIdx.x >> 6, l = threadIdx.x & 63;
  const long long pw = (long long)blockIdx.x * blockDim.x + (w << 6);  // first face of the wave
  const int nw = (int)min(64ll, (long long)L.tm.F - pw);               // faces of the wave
  uint32_t *lds = reinterpret_cast<uint32_t *>(stage[w]);
  {
    // face points of the four level-k children of p
    uint32_t v[12];
#pragma unroll
    for (int i = 0; i < 4; ++i) {
      v[3 * i + 0] = __float_as_uint(f[i].x);
      v[3 * i + 1] = __float_as_uint(f[i].y);
      v[3 * i + 2] = __float_as_uint(f[i].z);
    }
    wave_store<12>(lds, v, reinterpret_cast<uint32_t *>(L.P1 + 3ll * (Vk + 4 * pw)), l, 12 * nw);
  }
  if (L.fvk) {  // level-k face table: corners (v_i, EP(e_i), FP, EP(e_{i-1})) of child i
    uint32_t v[16];
#pragma unroll
    for (int i = 0; i < 4; ++i) {
      v[4 * i + 0] = cv[i];
      v[4 * i + 1] = VFm + e[i];
      v[4 * i + 2] = FP;
      v[4 * i + 3] = VFm + e[(i + 3) & 3];
    }
    wave_store<16>(lds, v, reinterpret_cast<uint32_t *>(L.fvk) + 16 * pw, l, 16 * nw);
  }
  if (L.ak.twin) {  // level-k twins and edge ids
    uint32_t v[16];
#pragma unroll
    for (int i = 0; i < 4; ++i) {
      const int ip = (i + 3) & 3;
      const int t = tw[i], tp = tw[ip];
      const int tn = t < 0 ? -1 : ((t & ~3) | ((t + 1) & 3));
      v[4 * i + 0] = t < 0 ? -1 : 4 * tn + 3;
      v[4 * i + 1] = 4 * (4 * p + ((i + 1) & 3)) + 2;
      v[4 * i + 2] = 4 * (4 * p + ip) + 1;
      v[4 * i + 3] = tp < 0 ? -1 : 4 * tp;
    }
    wave_store<16>(lds, v, reinterpret_cast<uint32_t *>(L.ak.twin) + 16 * pw, l, 16 * nw);
#pragma unroll
    for (int i = 0; i < 4; ++i)
#pragma unroll
      for (int r = 0; r < 4; ++r) v[4 * i + r] = kk[i][r];
    wave_store<16>(lds, v, reinterpret_cast<uint32_t *>(L.ak.eid) + 16 * pw, l, 16 * nw);
    if (valid) L.ak.vhe[FP] = 4 * (4 * p) + 2;
  }
  if (valid) {
    // vertex point of FP_m(p)
    const f3 sum = add3(add3(add3(pe[0], pe[1]), add3(pe[2], pe[3])), add3(add3(f[0], f[1]), add3(f[2], f[3])));
    st3(L.P1, FP, fma3(0.5f, pFP, mul3(1.0f / 16.0f, sum)));
  }
  if (L.fv1) {
    // the 16 children rows of level k+1 (256 B per face) as int4: the wave
    // stages all 16 rows of half its faces at a time (stride 17 int4 per
    // face) and stores them as 1 KB of contiguous rows per instruction
    // (4 faces x 16 rows). Staging 8 rows of all 64 faces (8 faces x 128 B
    // per instruction) was 2% slower, and 4 rows (half lines) 30% slower.
    int4 *o = reinterpret_cast<int4 *>(L.fv1);
    const int cc[4][4] = {{cv[0], VFm + e[0], FP, VFm + e[3]},
                          {cv[1], VFm + e[1], FP, VFm + e[0]},
                          {cv[2], VFm + e[2], FP, VFm + e[1]},
                          {cv[3], VFm + e[3], FP, VFm + e[2]}};
#pragma unroll
    for (int hf = 0; hf < 2; ++hf) {
      if ((l >> 5) == hf) {
#pragma unroll
        for (int x = 0; x < 16; ++x) {
          const int i = x >> 2, r = x & 3;
          stage[w][(l & 31) * 17 + x] = make_int4(cc[i][r], VFk + kk[i][r], Vk + 4 * p + i, VFk + kk[i][(r + 3) & 3]);
        }
      }
      __builtin_amdgcn_wave_barrier();
#pragma unroll
      for (int t = 0; t < 8; ++t) {
        const int g = 64 * t + l, fl = 32 * hf + (g >> 4);
        if (fl < nw) stream_store4(o + 16 * (pw + 32 * hf) + g, stage[w][(g >> 4) * 17 + (g & 15)]);
      }
      __builtin_amdgcn_wave_barrier();
    }
  }
  // ring terms of the level-m corners: edge point of the outgoing level-k edge + face point
  f3 term[4];
#pragma unroll
  for (int i = 0; i < 4; ++i) term[i] = add3(pe[i], f[i]);
  // corner 2: FP_g(pg), quad reduction over the siblings (symmetric tree)
  f3 r2 = add3(term[2], shfl_xor3(term[2], 1, 4));
  r2 = add3(r2, shfl_xor3(r2, 2, 4));
  // corner 1: EP_g(e_j) gets corner 3 of the next sibling
  const f3 t3n = shfl3(term[3], (j + 1) & 3, 4);
  const f3 pe3n = shfl3(pe[3], (j + 1) & 3, 4);
  if (!valid) return;
  if (j == 0) {
    st3(L.P1, cv[2], fma3(0.5f, pc[2], mul3(1.0f / 16.0f, r2)));
    if (L.ak.vhe) L.ak.vhe[cv[2]] = 4 * (4 * (4 * pg) + 2);
  }
  const f3 half = add3(term[1], t3n);
  if (tw[0] < 0) {
    // EP_g(e_j) on the boundary: 3/4 p + 1/8 (the two boundary neighbours at level k)
    st3(L.P1, cv[1], fma3(0.75f, pc[1], mul3(0.125f, add3(pe[0], pe3n))));
  } else {
    const int sg = tw[0] >> 4;  // grandparent quad across e_j
    const int eg = cv[1] - c.VFg;
    reinterpret_cast<f3 *>(c.hs)[2 * eg + (pg < sg ? 0 : 1)] = half;
  }
  // corner 0: a level-g vertex; its term is gathered by k_lag2_older
  reinterpret_cast<f3 *>(c.term0)[p] = term[0];
}

// edge points of level g (EP_g vertices): two half rings, crease valency
template <int BLK>
__global__ void __launch_bounds__(BLK) k_lag2_combine(Lag2Step c) {
  const int e = blockIdx.x * blockDim.x + threadIdx.x;
  if (e >= c.Eg) return;
  const LagStep &L = c.s;
  const int VFm = L.tm.V + L.tm.F;
  const int EPg = c.VFg + e;
  if (L.ak.vhe) L.ak.vhe[EPg] = 4 * L.am.vhe[EPg];
  const int bg = 4 * e - (L.bnd ? c.bscan_g[e] : 0);  // level-m halves of e: bg (lo end), bg + 1 (hi end)
  int kc = 0;
  double s0 = 0.0, s1 = 0.0;
  if (L.sigk) {
    const int x0 = lag_base(L, bg) + 1, x1 = lag_base(L, bg + 1) + 1;  // their level-k children at EP_g
    s0 = L.sigk[x0];
    s1 = L.sigk[x1];
    kc = (s0 > 0.0) + (s1 > 0.0);
    if (L.vcrk) L.vcrk[EPg] = make_int4(kc, s0 > 0.0 ? x0 : x1, kc == 2 ? x1 : -1, 0);
  }
  if (L.bnd && c.twin_g[c.e2h_g[e]] < 0) return;  // boundary: written by k_lag2_group
  const f3 *hs = reinterpret_cast<const f3 *>(c.hs);
  const f3 p = ld3(L.Pk, EPg);
  f3 S = fma3(0.5f, p, mul3(1.0f / 16.0f, add3(hs[2 * e], hs[2 * e + 1])));
  if (kc == 2) {
    const f3 sharp = fma3(0.75f, p, mul3(0.125f, add3(ld3(L.Pk, VFm + bg), ld3(L.Pk, VFm + bg + 1))));
    const double sv = (s0 + s1) * 0.5;
    if (sv >= 1.0) S = sharp;
    else {
      const float fs = (float)sv;
      S = fma3(1.0f - fs, S, mul3(fs, sharp));
    }
  }
  st3(L.P1, EPg, S);
}

// level-g vertices: the sum of the corner terms over their ring on level g.
// When level g was itself refined from quads, its face and interior edge
// points have their four ring half-edges in closed form, listed in the order
// the walk would visit them from the canonical start (so the sums are the
// same bits):
//   face point of quad p':  the slot-2 half-edges 16 p' + 2, + 6, + 10, + 14;
//   edge point of e' = (a, b): with a one of e''s half-edges whose child
//     carries the start, an = next(a), the twin of child a's slot 0 is slot 3
//     of child bn = next(b) on the other side: 4a+1, 4bn+3, 4b+1, 4an+3.
// Only the older vertices, and boundary edge points, walk.
__device__ __forceinline__ int quad_next(int h) { return (h & ~3) | ((h + 1) & 3); }
__device__ __forceinline__ int quad_prev(int h) { return (h & ~3) | ((h + 3) & 3); }

template <int BLK>
__global__ void __launch_bounds__(BLK) k_lag2_older(Lag2Step c) {
  const int v = blockIdx.x * blockDim.x + threadIdx.x;
  if (v >= c.Vg) return;
  const LagStep &L = c.s;
  const int VFm = L.tm.V + L.tm.F;
  const int h0 = c.vhe_g[v];
  const f3 *term0 = reinterpret_cast<const f3 *>(c.term0);
  const bool creases = L.sigk != nullptr;
  f3 sum{0.f, 0.f, 0.f};
  int n = 0, h = h0, hlast = h0;
  int kc = 0, cv0 = -1, cv1 = -1, ce0 = -1, ce1 = -1;
  double ssum = 0.0;
  bool bnd = false;
  // one incident level-m edge em = (v, EP_g): its level-k child at v has v as lower end
  auto crease = [&](int em) {
    const int x = lag_base(L, em);
    const double s = L.sigk[x];
    const bool on = s > 0.0;
    // selects, not branches: branches here were turned into a two-slot array
    // indexed by kc, which lived in scratch memory
    cv0 = (on && kc == 0) ? VFm + em : cv0;
    ce0 = (on && kc == 0) ? x : ce0;
    cv1 = (on && kc == 1) ? VFm + em : cv1;
    ce1 = (on && kc == 1) ? x : ce1;
    kc += on;
    ssum += on ? s : 0.0;
  };
  if (c.Vq > 0 && v >= c.Vq) {
    if (v < c.Vq + c.Fq) {  // face point: never on a crease or the boundary
      const int b = 16 * (v - c.Vq) + 2;
#pragma unroll
      for (int i = 0; i < 4; ++i) sum = add3(sum, term0[b + 4 * i]);
      n = 4;
      hlast = b + 12;
    } else {
      const int a = (h0 & 3) == 1 ? (h0 >> 2) : quad_prev(h0 >> 2);
      const int tw = c.twin_g[4 * a];
      if (tw >= 0) {  // interior edge point
        const int bn = tw >> 2, b = quad_prev(bn);
        const int cyc[4] = {4 * a + 1, 4 * bn + 3, 4 * b + 1, 4 * quad_next(a) + 3};
        // from the start: cyc[0..3], or cyc[3], cyc[0..2] (static indices: the
        // cycle stays in registers)
        const bool at0 = (h0 & 3) == 1;
#pragma unroll
        for (int j = 0; j < 4; ++j) {
          const int hj = at0 ? cyc[j] : cyc[(j + 3) & 3];
          sum = add3(sum, term0[hj]);
          if (creases) crease(L.am.eid[4 * hj]);
          hlast = hj;
        }
        n = 4;
      }
    }
  }
  if (n == 0) {
    // the fan first (only the twin loads in sequence), then every term at once
    constexpr int kFan = 8;
    int hs[kFan];
    bool go = true;
#pragma unroll
    for (int i = 0; i < kFan; ++i) {
      hs[i] = h;  // past the end: repeats the last half-edge (loads stay in bounds)
      if (go) {
        n = i + 1;
        const int t = c.twin_g[(h & 3) == 0 ? h + 3 : h - 1];
        if (t < 0) {
          bnd = true;
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
      for (int i = 0; i < kFan; ++i) tv[i] = term0[hs[i]];
#pragma unroll
      for (int i = 0; i < kFan; ++i)
        if (i < n) {
          sum = add3(sum, tv[i]);
          if (creases) crease(L.am.eid[4 * hs[i]]);
          hlast = hs[i];
        }
      if (creases && bnd) crease(L.am.eid[4 * hlast + 3]);  // the incoming boundary edge
    } else {  // a longer fan: walk it one step at a time
      n = 0;
      bnd = false;
      h = h0;
    }
  }
  if (n == 0) {
    while (true) {
      sum = add3(sum, term0[h]);
      ++n;
      hlast = h;
      if (creases) crease(L.am.eid[4 * h]);
      const int hp = (h & 3) == 0 ? h + 3 : h - 1;
      const int t = c.twin_g[hp];
      if (t < 0) {
        bnd = true;
        break;
      }
      if (t == h0 || n >= SUBDIV_MAX_VALENCE) break;
      h = t;
    }
    if (creases && bnd) crease(L.am.eid[4 * hlast + 3]);  // the incoming boundary edge
  }
  const f3 p = ld3(L.Pk, v);
  f3 S;
  if (bnd) {
    // boundary neighbours at level k: edge points of the level-m half-edges
    // v -> EP_g (corner 0 of child h0) and EP_g -> v (corner 3 of child hlast)
    const f3 b1 = ld3(L.Pk, VFm + L.am.eid[4 * h0]), b2 = ld3(L.Pk, VFm + L.am.eid[4 * hlast + 3]);
    S = fma3(0.75f, p, mul3(0.125f, add3(b1, b2)));
  } else {
    const float fn = (float)n;
    S = fma3(1.0f - 2.0f / fn, p, mul3(1.0f / (fn * fn), sum));
    if (kc >= 2) {
      const f3 sharp = (kc == 2) ? fma3(0.75f, p, mul3(0.125f, add3(ld3(L.Pk, cv0), ld3(L.Pk, cv1)))) : p;
      const double s = ssum / (double)kc;
      if (s >= 1.0) S = sharp;
      else {
        const float fs = (float)s;
        S = fma3(1.0f - fs, S, mul3(fs, sharp));
      }
    }
  }
  st3(L.P1, v, S);
  if (creases && L.vcrk) L.vcrk[v] = make_int4(kc, ce0, ce1, 0);
  if (L.ak.vhe) L.ak.vhe[v] = 16 * h0;
}

hipError_t lag2_launch(int which, const Lag2Step &c, hipStream_t s) {
  if (which == LAG2_GROUP)
    SUBDIV_LAUNCH_TUNED(TK_LAG2_GROUP, c.s.tm.F, s, k_lag2_group, c);
  else if (which == LAG2_COMBINE)
    SUBDIV_LAUNCH_TUNED(TK_LAG2_COMBINE, c.Eg, s, k_lag2_combine, c);
  else
    SUBDIV_LAUNCH_TUNED(TK_LAG2_OLDER, c.Vg, s, k_lag2_older, c);
  return hipGetLastError();
}

}  // namespace subdiv
