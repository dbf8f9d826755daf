// Loop (App. B) and sqrt(3) (App. A) level steps on gfx950. Both use the
// adjacency of the same level from the generic build: twin half-edges give
// G(i,j)/G(j,i) (the opposite vertices, Loop) and F(l,k) (the neighbouring
// face, sqrt(3)); edge ids come from the upper triangle of E.
//
// Loop:   edge point 3/8 (p_a + p_b) + 1/8 (p_c + p_d), boundary midpoint;
//         vertex (1 - n beta_n) p + beta_n sum p_j (eq:loop_smooth), boundary
//         3/4 p + 1/8 (p_prev + p_next); children 4r+j (j<3) =
//         (v_j, e(j,j+1), e(j-1,j)), 4r+3 = (e01, e12, e20).
// sqrt3:  face point mapped M^T P with (1,2,3) -> 1/3; vertex
//         (1 - alpha_n) p + alpha_n / n sum p_j (equ:sqrt2, equ:alpha), boundary
//         vertices fixed; child 3r+j = (v_j, face across edge j, face r) or
//         (v_j, v_j+1, face r) on a boundary edge (the face point of face i has
//         index |v| + i).
// beta_n and alpha_n are evaluated once on the host in FP64 and rounded to
// FP32 into constant memory: no device cosine decides a weight.
#include <climits>
#include <cmath>
#include <mutex>

#include "subdiv_internal.h"

namespace subdiv {

__constant__ float c_loop_beta[SUBDIV_MAX_VALENCE + 1];
__constant__ float c_sqrt3_alpha[SUBDIV_MAX_VALENCE + 1];

hipError_t init_weight_tables() {
  static std::mutex mu;
  static int done_device = -1;
  std::lock_guard<std::mutex> lock(mu);
  int dev = 0;
  hipError_t err = hipGetDevice(&dev);
  if (err != hipSuccess) return err;
  if (done_device == dev) return hipSuccess;
  static float beta[SUBDIV_MAX_VALENCE + 1], alpha[SUBDIV_MAX_VALENCE + 1];
  const double pi = 3.14159265358979323846;
  beta[0] = alpha[0] = 0.f;
  for (int n = 1; n <= SUBDIV_MAX_VALENCE; ++n) {
    const double c = 3.0 / 8.0 + 0.25 * std::cos(2.0 * pi / n);
    beta[n] = (float)((5.0 / 8.0 - c * c) / n);
    alpha[n] = (float)((4.0 - 2.0 * std::cos(2.0 * pi / n)) / 9.0);
  }
  if ((err = hipMemcpyToSymbol(HIP_SYMBOL(c_loop_beta), beta, sizeof(beta))) != hipSuccess) return err;
  if ((err = hipMemcpyToSymbol(HIP_SYMBOL(c_sqrt3_alpha), alpha, sizeof(alpha))) != hipSuccess) return err;
  done_device = dev;
  return hipSuccess;
}

// Loop's edge-point stencil and the stencils of the vertex points of edge
// points, with every product and sum rounded on its own: the pragma keeps
// the compiler from fusing them into multiply-adds, whose placement it picks
// per kernel. The per-level kernels and the last step from two levels down
// evaluate them from different index paths and give the same bits.
__device__ __forceinline__ f3 lin2(float s, f3 a, float t, f3 b) {
#pragma clang fp contract(off)
  return f3{s * a.x + t * b.x, s * a.y + t * b.y, s * a.z + t * b.z};
}
// 3/8 (sum of the edge's ends) + 1/8 (sum of the opposite corners)
__device__ __forceinline__ f3 loop_edge_pt(f3 ends, f3 opp) { return lin2(0.375f, ends, 0.125f, opp); }
// boundary vertex: 3/4 p + 1/8 (sum of its two boundary neighbours)
__device__ __forceinline__ f3 loop_bnd_pt(f3 p, f3 nb) { return lin2(0.75f, p, 0.125f, nb); }
// interior vertex of valence 6 (every edge point of a refined level)
__device__ __forceinline__ f3 loop_v6_pt(f3 p, f3 ring) {
#pragma clang fp contract(off)
  const float beta = c_loop_beta[6];
  return lin2(1.0f - 6.0f * beta, p, beta, ring);
}
// interior vertex of valence n: (1 - n beta_n) p + beta_n (sum of the ring),
// the ring summed in the order of the walk from the vertex's start
__device__ __forceinline__ f3 loop_old_pt(f3 p, f3 ring, int n) {
#pragma clang fp contract(off)
  const float beta = c_loop_beta[n];
  return lin2(1.0f - (float)n * beta, p, beta, ring);
}
__device__ __forceinline__ f3 sel3(bool c, f3 a, f3 b) { return c ? a : b; }

// sqrt(3) interior vertex: (1 - alpha_n) p + alpha_n / n (sum of the n
// neighbours), uncontracted like the Loop stencils (the face point of a
// refined level is evaluated by two kernels)
__device__ __forceinline__ f3 sqrt3_pt(f3 p, f3 ring, int n) {
#pragma clang fp contract(off)
  const float alpha = c_sqrt3_alpha[n];
  return lin2(1.0f - alpha, p, alpha / (float)n, ring);
}

// a_j for a runtime j in 0..2, by selects (a dynamic index into an array
// would put the array in scratch memory)
__device__ __forceinline__ int pick3(int a0, int a1, int a2, int j) { return j == 0 ? a0 : j == 1 ? a1 : a2; }

// s + a + b + c + d + e + f, added in that order (a ring sum from its start)
__device__ __forceinline__ f3 sum6(f3 s, f3 a, f3 b, f3 c, f3 d, f3 e, f3 f) {
  s = add3(s, a);
  s = add3(s, b);
  s = add3(s, c);
  s = add3(s, d);
  s = add3(s, e);
  return add3(s, f);
}

// ring walk around v: sum of the neighbours, count of faces, boundary ends
struct Ring {
  f3 sum;
  int faces;
  int w0;  // end of the first half-edge (boundary neighbour if on the boundary)
  int ub;  // start of the last incoming boundary half-edge, -1 if interior
};

// The fan of half-edges leaving a vertex, from h0 in rotation order, up to
// kFan of them: only the dependent twin loads run in sequence here, and the
// caller then issues every neighbour gather at once. Returns the count, or -1
// when the fan is longer (the caller walks it one step at a time); hb = the
// last half-edge when the fan ends at the boundary, else -1. Entries past the
// count repeat the last half-edge, so loads through them stay in bounds.
constexpr int kFan = 8;
__device__ __forceinline__ int fan3(const int32_t *twin, int h0, int (&hs)[kFan], int &hb) {
  int n = 0, h = h0;
  bool go = true;
  hb = -1;
#pragma unroll
  for (int i = 0; i < kFan; ++i) {
    hs[i] = h;
    if (go) {
      n = i + 1;
      const int tw = twin[h % 3 == 0 ? h + 2 : h - 1];
      if (tw < 0) {
        hb = h;
        go = false;
      } else if (tw == h0) {
        go = false;
      } else {
        h = tw;
      }
    }
  }
  return go ? -1 : n;
}

__device__ __forceinline__ Ring ring3(const Topo &t, const Adj &a, const float *P, int v) {
  const int h0 = a.vhe[v];
  Ring R{{0.f, 0.f, 0.f}, 0, t.fv[he_next<3>(t, h0)], -1};
  int h = h0;
  while (true) {
    R.sum = add3(R.sum, ld3(P, t.fv[he_next<3>(t, h)]));
    ++R.faces;
    const int hp = he_prev<3>(t, h);
    const int tw = a.twin[hp];
    if (tw < 0) {
      R.ub = t.fv[hp];
      R.sum = add3(R.sum, ld3(P, R.ub));
      break;
    }
    if (tw == h0 || R.faces >= SUBDIV_MAX_VALENCE) break;
    h = tw;
  }
  return R;
}

// The point born from face r of the level below (a face point, or p of the
// trisection step) whose three child rows read (v_i, X_i, point), every X_i a
// new point: its ring on its own level is v_0, X_0, v_1, X_1, v_2, X_2 around
// from the start (the least of the half-edges point -> v_i = 9r + 3i + 2 and
// point -> X_i = twin of slot 1 of child i), the order of the walk. Faces next
// to the boundary (an X_i that is a corner, or other rows) are walked.
__device__ __forceinline__ bool ring_rows_fp(const Topo &t, const Adj &a, const float *P, int v, int r, Ring &R) {
  const int32_t *rw = t.fv + 9ll * r;
  int x[9];
#pragma unroll
  for (int i = 0; i < 9; ++i) x[i] = rw[i];
  if (x[2] != v || x[5] != v || x[8] != v || x[1] < v - r || x[4] < v - r || x[7] < v - r) return false;
  const int h0 = a.vhe[v];
  const int32_t *tr = a.twin + 9ll * r;
  int p0 = 0;
#pragma unroll
  for (int i = 0; i < 3; ++i)
    if (tr[3 * i + 1] == h0) p0 = 2 * i + 1;
  f3 pt[6];
#pragma unroll
  for (int y = 0; y < 6; ++y) pt[y] = ld3(P, x[3 * (y >> 1) + (y & 1)]);
  // (the rotation by cases, so that pt stays in registers)
  if (p0 == 1) R.sum = sum6(R.sum, pt[1], pt[2], pt[3], pt[4], pt[5], pt[0]);
  else if (p0 == 3) R.sum = sum6(R.sum, pt[3], pt[4], pt[5], pt[0], pt[1], pt[2]);
  else if (p0 == 5) R.sum = sum6(R.sum, pt[5], pt[0], pt[1], pt[2], pt[3], pt[4]);
  else R.sum = sum6(R.sum, pt[0], pt[1], pt[2], pt[3], pt[4], pt[5]);
  R.faces = 6;
  return true;
}

// An interior old vertex v of a level k made by a trisection step has one
// neighbour per level-(k-1) face s_i around it, in the order of its fan
// there (g_i the half-edge leaving v in s_i): the point of the face s_{i-1}
// before s_i toward s_i (its q when s_i lies across the edge after its
// boundary edge, else its face point or p), followed by p_i itself when v is
// the apex of the boundary face s_i (opposite its boundary edge j). Those
// entries come from the half-edges 3 g_i and 9 s_i + 3 j + 2 of level k, and
// the walk starts at the least of them. So the ring is read from level k-1's
// fan, a third of level k's rows. Boundary vertices are fixed.
__device__ __forceinline__ bool ring_trisected_old(const TriStep &c, int v, Ring &R) {
  const Adj &x = c.ap;
  const int g0 = x.vhe[v];
  int gs[kFan], hb;
  const int n = fan3(x.twin, g0, gs, hb);
  if (n < 0) return false;  // a longer fan: walked on level k
  if (hb >= 0) {  // on the boundary: the vertex stays where it is
    R.faces = n;
    R.ub = 0;
    return true;
  }
  const int Vp = c.fpV, Fp = c.fpF;
  int glast = gs[0];
#pragma unroll
  for (int i = 0; i < kFan; ++i)
    if (i < n) glast = gs[i];
  int sl[kFan];
#pragma unroll
  for (int i = 0; i < kFan; ++i) sl[i] = c.pbslot[gs[i] / 3];
  int nb[2 * kFan], key[2 * kFan];
  bool ok[2 * kFan];
#pragma unroll
  for (int i = 0; i < kFan; ++i) {
    const int gp = i == 0 ? glast : gs[i - 1], sp = gp / 3;
    const int jp = i == 0 ? c.pbslot[sp] : sl[i - 1];
    const bool q = jp >= 0 && (gp % 3 + 2) % 3 == (jp + 1) % 3;  // s_i lies across sp's edge after its boundary edge
    nb[2 * i] = q ? Vp + Fp + c.pbrank[sp] : Vp + sp;
    key[2 * i] = 3 * gs[i];
    ok[2 * i] = i < n;
    const int si = gs[i] / 3, j = sl[i];
    ok[2 * i + 1] = i < n && j >= 0 && gs[i] % 3 == (j + 2) % 3;
    nb[2 * i + 1] = Vp + si;
    key[2 * i + 1] = 9 * si + 3 * j + 2;
  }
  int st = 0, best = key[0];
#pragma unroll
  for (int e = 1; e < 2 * kFan; ++e)
    if (ok[e] && key[e] < best) {
      best = key[e];
      st = e;
    }
  f3 pt[2 * kFan];
#pragma unroll
  for (int e = 0; e < 2 * kFan; ++e) pt[e] = ld3(c.P, ok[e] ? nb[e] : v);
  int m = 0;
#pragma unroll
  for (int e = 0; e < 2 * kFan; ++e)
    if (ok[e] && e >= st) {
      R.sum = add3(R.sum, pt[e]);
      ++m;
    }
#pragma unroll
  for (int e = 0; e < 2 * kFan; ++e)
    if (ok[e] && e < st) {
      R.sum = add3(R.sum, pt[e]);
      ++m;
    }
  R.faces = m;
  R.ub = -1;
  return true;
}

// The old vertices v < Vg of a refined level k keep their rings from level
// k-1: their level-k half-edges are the first slots of the children at their
// level-(k-1) half-edges, in the same rotation order, and the neighbour along
// each is a point of level k named by that level-(k-1) half-edge (Loop: the
// edge point Vg + eid; sqrt(3): the face point Vg + face across it). So the
// ring is walked on level k-1, whose rows are a third or a quarter as many,
// visiting the same neighbours in the same order (the sums are the same
// bits). sqrt(3) fixes boundary vertices, so there only the boundary test is
// kept (the same half-edges end the walk on both levels).
//
// One level further down, an old vertex that was itself new on level k-1
// has its level-(k-1) ring in closed form, listed here in walk order from its
// canonical start (so again the same bits):
//   Loop, edge point u of edge j of face r (edge i of the face s across): the
//     six half-edges slot 1 of child j of r, slot 2 of child i+1 of s, slot i
//     of s's centre child, slot 1 of child i of s, slot 2 of child j+1 of r,
//     slot j of r's centre child (h1(q, slot) = 3 q + slot, children 4 r + c);
//     the start is the first of these or the fifth;
//   sqrt(3), face point of face r: slot 2 of r's child j (F_r -> v_j) and the
//     twin of slot 1 of that child (F_r -> F_s in the child of the face s
//     across edge j), alternating over j; the start is slot 2 of child 0 or
//     one of those twins. Only interior edge / face points take this form.
__device__ __forceinline__ Ring ring_prev_loop(const TriStep &c, int v) {
  const Adj &a = c.ap;
  const int h0 = a.vhe[v];
  Ring R{{0.f, 0.f, 0.f}, 0, c.Vg + a.eid[h0], -1};
  if (c.Vq > 0 && v >= c.Vq) {
    const int q = h0 / 3, r = q >> 2, cq = q & 3;
    const bool first = (h0 % 3 == 1);  // else slot 2 of child j+1
    const int j = first ? cq : (cq + 2) % 3;
    const int tw = a.twin[12 * r + 3 * j];  // v_j -> E_j: slot 2 of child i+1 of s
    if (tw >= 0) {
      const int qs = tw / 3, s = qs >> 2, i = ((qs & 3) + 2) % 3;
      const int jn = (j + 1) % 3, in = (i + 1) % 3;
      const int cyc[6] = {12 * r + 3 * j + 1, 12 * s + 3 * in + 2, 12 * s + 9 + i,
                          12 * s + 3 * i + 1, 12 * r + 3 * jn + 2, 12 * r + 9 + j};
      const int p0 = first ? 0 : 4;
#pragma unroll
      for (int t = 0; t < 6; ++t) {
        const int x = p0 + t;
        R.sum = add3(R.sum, ld3(c.P, c.Vg + a.eid[cyc[x < 6 ? x : x - 6]]));
      }
      R.faces = 6;
      return R;
    }
  }
  int hs[kFan], hb;
  const int n = fan3(a.twin, h0, hs, hb);
  if (n > 0) {
    f3 pt[kFan];
#pragma unroll
    for (int i = 0; i < kFan; ++i) pt[i] = ld3(c.P, c.Vg + a.eid[hs[i]]);
#pragma unroll
    for (int i = 0; i < kFan; ++i)
      if (i < n) R.sum = add3(R.sum, pt[i]);
    R.faces = n;
    if (hb >= 0) {
      R.ub = c.Vg + a.eid[he_prev<3>(c.t, hb)];
      R.sum = add3(R.sum, ld3(c.P, R.ub));
    }
    return R;
  }
  int h = h0;
  while (true) {
    R.sum = add3(R.sum, ld3(c.P, c.Vg + a.eid[h]));
    ++R.faces;
    const int hp = he_prev<3>(c.t, h);
    const int tw = a.twin[hp];
    if (tw < 0) {
      R.ub = c.Vg + a.eid[hp];
      R.sum = add3(R.sum, ld3(c.P, R.ub));
      break;
    }
    if (tw == h0 || R.faces >= SUBDIV_MAX_VALENCE) break;
    h = tw;
  }
  return R;
}

// The walk itself: the ring of an old vertex of a level refined by a sqrt(3)
// step from the level with adjacency a, walked there from the vertex's start
// h0: the neighbour across each half-edge is the face point Vg + (the face
// of its twin).
__device__ __forceinline__ void walk_below_sqrt3(const Adj &a, const float *P, int Vg, int h0, Ring &R) {
  int hs[kFan], hb;
  const int n = fan3(a.twin, h0, hs, hb);
  if (n > 0) {
    int ts[kFan];
    f3 pt[kFan];
#pragma unroll
    for (int i = 0; i < kFan; ++i) ts[i] = a.twin[hs[i]];
#pragma unroll
    for (int i = 0; i < kFan; ++i) pt[i] = ld3(P, Vg + (ts[i] >= 0 ? ts[i] / 3 : 0));
#pragma unroll
    for (int i = 0; i < kFan; ++i)
      if (i < n && ts[i] >= 0) R.sum = add3(R.sum, pt[i]);
    R.faces = n;
    R.ub = hb >= 0 ? 0 : -1;  // on the boundary: the vertex stays where it is
    return;
  }
  // (every exit writes both counts: a store to one of them on some paths
  // only makes the compiler keep the ring in scratch memory)
  int h = h0, nf = R.faces, ub = -1;
  while (true) {
    const int ts = a.twin[h];
    if (ts >= 0) R.sum = add3(R.sum, ld3(P, Vg + ts / 3));
    ++nf;
    const int tw = a.twin[h % 3 == 0 ? h + 2 : h - 1];
    if (tw < 0) {
      ub = 0;  // on the boundary: the vertex stays where it is
      break;
    }
    if (tw == h0 || nf >= SUBDIV_MAX_VALENCE) break;
    h = tw;
  }
  R.faces = nf;
  R.ub = ub;
}

__device__ __forceinline__ Ring ring_prev_sqrt3(const TriStep &c, int v) {
  const Adj &a = c.ap;
  const int h0 = a.vhe[v];
  Ring R{{0.f, 0.f, 0.f}, 0, 0, -1};
  if (c.Vq > 0 && v >= c.Vq) {
    const int r = v - c.Vq;
    const int *tr = a.twin + 9ll * r;
    const int t1[3] = {tr[1], tr[4], tr[7]}, t2[3] = {tr[2], tr[5], tr[8]};
    // slot 1 of a child whose edge is interior pairs with slot 1 of the child of s
    if (t1[0] % 3 == 1 && t1[1] % 3 == 1 && t1[2] % 3 == 1) {
      int p0 = 0;
#pragma unroll
      for (int j = 0; j < 3; ++j)
        if (h0 == t1[j]) p0 = 2 * j + 1;
#pragma unroll
      for (int t = 0; t < 6; ++t) {
        const int x = p0 + t < 6 ? p0 + t : p0 + t - 6, j = x >> 1;
        // across F_r -> v_j: the face holding v_j -> F_r; across F_r -> F_s: r's child j
        const int face = (x & 1) ? 3 * r + j : pick3(t2[0], t2[1], t2[2], j) / 3;
        R.sum = add3(R.sum, ld3(c.P, c.Vg + face));
      }
      R.faces = 6;
      return R;
    }
  }
  walk_below_sqrt3(a, c.P, c.Vg, h0, R);
  return R;
}

// Two levels down. An old vertex v < V_{k-2} of level k has the same ring
// on level k-2, k-1 and k: the first-slot map takes a half-edge leaving v on
// one level to the half-edge leaving v in the child at it on the next (Loop
// h -> 4h - h mod 3, sqrt(3) h -> 3h), keeping the rotation order and the
// boundary. So the walk (and, for the points born on level k-2, the closed
// form) runs on level k-2's rows, a sixteenth (a ninth) of level k's, and
// only the neighbour lookups touch level k-1: along the image h' of h the
// neighbour is the level-k point named by h' (Loop: Vg + eid(h'); sqrt(3):
// the face point Vg + (face across h')). Same neighbours, same order, same
// bits as the walk one level down.
__device__ __forceinline__ Ring ring_prev2_loop(const TriStep &c, int v) {
  const Adj &x = c.app;
  const int32_t *eid1 = c.ap.eid;
  auto nb = [&](int h) { return c.Vg + eid1[4 * h - h % 3]; };
  const int h0 = x.vhe[v];
  Ring R{{0.f, 0.f, 0.f}, 0, nb(h0), -1};
  if (c.Vr > 0 && v >= c.Vr) {
    const int q = h0 / 3, r = q >> 2, cq = q & 3;
    const bool first = (h0 % 3 == 1);
    const int j = first ? cq : (cq + 2) % 3;
    const int tw = x.twin[12 * r + 3 * j];
    if (tw >= 0) {
      const int qs = tw / 3, s = qs >> 2, i = ((qs & 3) + 2) % 3;
      const int jn = (j + 1) % 3, in = (i + 1) % 3;
      const int cyc[6] = {12 * r + 3 * j + 1, 12 * s + 3 * in + 2, 12 * s + 9 + i,
                          12 * s + 3 * i + 1, 12 * r + 3 * jn + 2, 12 * r + 9 + j};
      const int p0 = first ? 0 : 4;
#pragma unroll
      for (int t = 0; t < 6; ++t) {
        const int y = p0 + t;
        R.sum = add3(R.sum, ld3(c.P, nb(cyc[y < 6 ? y : y - 6])));
      }
      R.faces = 6;
      return R;
    }
  }
  int hs[kFan], hb;
  const int n = fan3(x.twin, h0, hs, hb);
  if (n > 0) {
    f3 pt[kFan];
#pragma unroll
    for (int i = 0; i < kFan; ++i) pt[i] = ld3(c.P, nb(hs[i]));
#pragma unroll
    for (int i = 0; i < kFan; ++i)
      if (i < n) R.sum = add3(R.sum, pt[i]);
    R.faces = n;
    if (hb >= 0) {
      R.ub = c.Vg + eid1[4 * hb - hb % 3 + 2];
      R.sum = add3(R.sum, ld3(c.P, R.ub));
    }
    return R;
  }
  int h = h0;
  while (true) {
    R.sum = add3(R.sum, ld3(c.P, nb(h)));
    ++R.faces;
    const int hp = he_prev<3>(c.t, h);
    const int tw = x.twin[hp];
    if (tw < 0) {
      R.ub = c.Vg + eid1[4 * h - h % 3 + 2];  // the incoming half-edge of the child at h
      R.sum = add3(R.sum, ld3(c.P, R.ub));
      break;
    }
    if (tw == h0 || R.faces >= SUBDIV_MAX_VALENCE) break;
    h = tw;
  }
  return R;
}

// sqrt(3) needs no lookup on level k-1 at all: the image of an interior
// half-edge h of level k-2 is the first slot 3h of the child at h, whose twin
// is slot 2 of the child at v of the face s across h (h's twin t = 3s + i,
// that child 3s + (i+1) mod 3), so the face point across the image is
// Vg + 3 (t / 3) + (t mod 3 + 1) mod 3, from the twin on level k-2 alone.
__device__ __forceinline__ int sqrt3_across_image(int t) { return 3 * (t / 3) + (t % 3 + 1) % 3; }

// The rings of the cage's vertices and of its face points from the cage's
// adjacency (twice as many ints as cage faces: it stays in L2) rather than a
// walk on level l: repeating the map above, a half-edge of level b with twin
// t = 3s + i has on level l > b the image across from the face
// 3^(l-b-1) (3s + (i+1) mod 3). A cage vertex (b = 0) walks its cage fan. The
// face point of cage face r (b = 1, l >= 2) has the six-half-edge ring of the
// closed form above, starting at the least of them; the twins of its
// half-edges on level 1 follow from r's three cage twins (t2 of the edge
// before, 9r + 3j + 1). Same neighbours in the same order as the walks.
__device__ __forceinline__ bool ring_cage_sqrt3(const TriStep &c, int v, Ring &R) {
  const int32_t *tw0 = c.a0.twin;
  if (v < c.V0) {
    const int m0 = c.pow3;
    const int h0 = c.a0.vhe[v];
    int hs[kFan], hb;
    const int n = fan3(tw0, h0, hs, hb);
    if (n > 0) {
      R.faces = n;
      if (hb >= 0) {  // on the boundary: the vertex stays where it is
        R.ub = 0;
        return true;
      }
      int ts[kFan];
      f3 pt[kFan];
#pragma unroll
      for (int i = 0; i < kFan; ++i) ts[i] = tw0[hs[i]];
#pragma unroll
      for (int i = 0; i < kFan; ++i) pt[i] = ld3(c.P, c.Vg + m0 * sqrt3_across_image(ts[i]));
#pragma unroll
      for (int i = 0; i < kFan; ++i)
        if (i < n) R.sum = add3(R.sum, pt[i]);
      R.ub = -1;
      return true;
    }
    int h = h0, nf = R.faces, ub = -1;
    while (true) {
      const int ts = tw0[h];
      if (ts >= 0) R.sum = add3(R.sum, ld3(c.P, c.Vg + m0 * sqrt3_across_image(ts)));
      ++nf;
      const int tw = tw0[h % 3 == 0 ? h + 2 : h - 1];
      if (tw < 0) {
        ub = 0;
        break;
      }
      if (tw == h0 || nf >= SUBDIV_MAX_VALENCE) break;
      h = tw;
    }
    R.faces = nf;
    R.ub = ub;
    return true;
  }
  if (c.pow3 >= 3 && v < c.V0 + c.F0) {
    const int r = v - c.V0;
    const int t[3] = {tw0[3 * r], tw0[3 * r + 1], tw0[3 * r + 2]};
    if (t[0] < 0 || t[1] < 0 || t[2] < 0) return false;  // next to the boundary: walked
    int p0 = 0, best = 9 * r + 2;
#pragma unroll
    for (int j = 0; j < 3; ++j) {
      const int t1 = 9 * (t[j] / 3) + 3 * (t[j] % 3) + 1;  // F_r -> F_s on level 1
      if (t1 < best) {
        best = t1;
        p0 = 2 * j + 1;
      }
    }
    const int m1 = c.pow3 / 3;
#pragma unroll
    for (int u = 0; u < 6; ++u) {
      const int y = p0 + u < 6 ? p0 + u : p0 + u - 6, j = y >> 1, tp = pick3(t[0], t[1], t[2], (j + 2) % 3);
      const int T = (y & 1) ? 9 * r + 3 * j + 1 : 9 * (tp / 3) + 3 * (tp % 3);
      R.sum = add3(R.sum, ld3(c.P, c.Vg + m1 * sqrt3_across_image(T)));
    }
    R.faces = 6;
    R.ub = -1;
    return true;
  }
  return false;
}

__device__ __forceinline__ Ring ring_prev2_sqrt3(const TriStep &c, int v) {
  const Adj &x = c.app;
  const int h0 = x.vhe[v];
  Ring R{{0.f, 0.f, 0.f}, 0, 0, -1};
  if (c.Vr > 0 && v >= c.Vr) {
    const int r = v - c.Vr;
    const int *tr = x.twin + 9ll * r;
    const int t1[3] = {tr[1], tr[4], tr[7]}, t2[3] = {tr[2], tr[5], tr[8]};
    if (t1[0] % 3 == 1 && t1[1] % 3 == 1 && t1[2] % 3 == 1) {
      int p0 = 0;
#pragma unroll
      for (int j = 0; j < 3; ++j)
        if (h0 == t1[j]) p0 = 2 * j + 1;
#pragma unroll
      for (int t = 0; t < 6; ++t) {
        const int y = p0 + t < 6 ? p0 + t : p0 + t - 6, j = y >> 1;
        // the ring's half-edges alternate F_r -> v_j (slot 2 of r's child j,
        // twin t2[j]) and F_r -> F_s (t1[j], the twin of r's child j's slot
        // 1); all interior
        const int tw = (y & 1) ? 9 * r + 3 * j + 1 : pick3(t2[0], t2[1], t2[2], j);
        R.sum = add3(R.sum, ld3(c.P, c.Vg + sqrt3_across_image(tw)));
      }
      R.faces = 6;
      R.ub = -1;
      return R;
    }
  }
  int hs[kFan], hb;
  const int n = fan3(x.twin, h0, hs, hb);
  if (n > 0) {
    if (hb >= 0) {  // on the boundary: the vertex stays where it is
      R.faces = n;
      R.ub = 0;
      return R;
    }
    int ts[kFan];
    f3 pt[kFan];
#pragma unroll
    for (int i = 0; i < kFan; ++i) ts[i] = x.twin[hs[i]];  // (the row the fan step just read)
#pragma unroll
    for (int i = 0; i < kFan; ++i) pt[i] = ld3(c.P, c.Vg + sqrt3_across_image(ts[i]));
#pragma unroll
    for (int i = 0; i < kFan; ++i)
      if (i < n) R.sum = add3(R.sum, pt[i]);
    R.faces = n;
    R.ub = -1;
    return R;
  }
  int h = h0, nf = 0, ub = -1;
  while (true) {
    const int ts = x.twin[h];
    if (ts >= 0) R.sum = add3(R.sum, ld3(c.P, c.Vg + sqrt3_across_image(ts)));
    ++nf;
    const int tw = x.twin[he_prev<3>(c.t, h)];
    if (tw < 0) {
      ub = 0;  // on the boundary: the vertex stays where it is
      break;
    }
    if (tw == h0 || nf >= SUBDIV_MAX_VALENCE) break;
    h = tw;
  }
  R.faces = nf;
  R.ub = ub;
  return R;
}

// ------------------------------------------------------------------ Loop
// Carried adjacency of the next level (App. B topology: children 4r+j, j<3,
// = (v_j, E_j, E_{j-1}) and 4r+3 = (E_0, E_1, E_2), E_j = |v| + e_j).
// Every edge of level k+1 has an edge point E_e as its higher end; its lower
// neighbours, ascending, are lo(e), hi(e) and the edge points E_e' of the
// edges e' < e that share a face with e (the set N(e), at most four). So the
// edges with higher end E_e take ids base(e) .. base(e) + 1 + |{e' in N(e),
// e' < e}|, base = exclusive scan of those counts over e, and
//   (lo(e), E_e) -> base(e), (hi(e), E_e) -> base(e) + 1,
//   (E_a, E_b), a < b -> base(b) + 2 + |{e' in N(b), e' < a}|.
// N(e) is counted as a set (two faces may share more than one edge).
__device__ __forceinline__ int lt_new(int x, int bound, int o1, int o2) {
  return (x < bound && x != o1 && x != o2) ? 1 : 0;
}

template <int BLK>
__global__ void __launch_bounds__(BLK) k_loop_edge(TriStep c) {
  const int e = blockIdx.x * blockDim.x + threadIdx.x;
  if (e >= c.a.E) return;
  const int h = c.a.e2h[e];
  const int hn = he_next<3>(c.t, h), hp = he_prev<3>(c.t, h);
  const int t = c.a.twin[h];
  if (c.P1) {  // (without P1: only the counts, the points come from the level below)
    const f3 pab = add3(ld3(c.P, c.t.fv[h]), ld3(c.P, c.t.fv[hn]));
    f3 ep;
    if (t < 0) ep = mul3(0.5f, pab);
    else {
      const f3 pcd = add3(ld3(c.P, c.t.fv[hp]), ld3(c.P, c.t.fv[he_prev<3>(c.t, t)]));
      ep = loop_edge_pt(pab, pcd);
    }
    if (t >= 0 && c.a.sig) {  // a crease edge: Loop's edge point blended with the midpoint
      const double sg = c.a.sig[e];
      if (sg >= 1.0) {
        ep = mul3(0.5f, pab);
      } else if (sg > 0.0) {
        const float w = (float)sg;
        ep = lin2(1.0f - w, ep, 0.5f * w, pab);
      }
    }
    st3(c.P1, c.t.V + e, ep);
  }
  if (c.base) {  // children of level k+1 with higher end E_e
    const int n1 = c.a.eid[hn], n2 = c.a.eid[hp];
    int cnt = 2 + (n1 < e) + (n2 < e);
    if (t >= 0) {
      cnt += lt_new(c.a.eid[he_next<3>(c.t, t)], e, n1, n2);
      cnt += lt_new(c.a.eid[he_prev<3>(c.t, t)], e, n1, n2);
    }
    c.base[e] = cnt;
  }
}

// Edge-point vertex u = Vg + e of a refined level k: its ring lies in the
// children of the two level-(k-1) faces of e. Its canonical half-edge
// (the lowest outgoing one, or the boundary one) sits in the children of the
// face r owning e and names e's slot j there; r's child rows hold v_j,
// v_{j+1} and the edge points of r's other edges, the twin of v_j -> E_j
// names the face s across e, whose centre child holds the other two.
__device__ __forceinline__ f3 loop_ep_point(const TriStep &c, int u) {
  const f3 p = ld3(c.P, u);
  const int h0 = c.a.vhe[u], q = h0 / 3, r = q >> 2, cq = q & 3;
  const int j = (h0 % 3 == 1) ? cq : (cq + 2) % 3;  // E_j -> E_{j-1} in child j, or E_j -> v_{j+1} in child j+1
  const int jn = (j + 1) % 3, jp = (j + 2) % 3;
  const int32_t *rw = c.t.fv + 12ll * r;
  const f3 pa = ld3(c.P, rw[3 * j]), pb = ld3(c.P, rw[3 * jn]);
  const int tw = c.a.twin[12 * r + 3 * j];  // twin of v_j -> E_j
  if (tw < 0) return loop_bnd_pt(p, add3(pa, pb));
  const f3 n1 = ld3(c.P, rw[9 + jn]), n2 = ld3(c.P, rw[9 + jp]);
  const int qs = tw / 3, s = qs >> 2, i = ((qs & 3) + 2) % 3;  // e is edge i of s
  const int32_t *sw = c.t.fv + 12ll * s + 9;
  const f3 x = ld3(c.P, sw[(i + 1) % 3]), y = ld3(c.P, sw[(i + 2) % 3]);
  return loop_v6_pt(p, add3(add3(pa, pb), add3(add3(n1, n2), add3(x, y))));
}

template <int BLK>
__global__ void __launch_bounds__(BLK) k_loop_vertex(TriStep c) {
  const int v = blockIdx.x * blockDim.x + threadIdx.x;
  if (v >= c.t.V) return;
  if (c.Vg > 0 && v >= c.Vg) {  // an edge point of the previous level: no ring walk
    st3(c.P1, v, loop_ep_point(c, v));
    if (c.a1.vhe) {
      const int h0 = c.a.vhe[v];
      c.a1.vhe[v] = 4 * h0 - h0 % 3;
    }
    return;
  }
  const f3 p = ld3(c.P, v);
  const Ring R = c.Vg == 0                     ? ring3(c.t, c.a, c.P, v)
                 : (c.app.twin && v < c.Vq) ? ring_prev2_loop(c, v)
                                            : ring_prev_loop(c, v);
  const f3 S = R.ub >= 0 ? loop_bnd_pt(p, add3(ld3(c.P, R.w0), ld3(c.P, R.ub))) : loop_old_pt(p, R.sum, R.faces);
  st3(c.P1, v, S);
  // an old vertex's half-edges at level k+1 are the first halves 3 (4r + j)
  // of its level-k half-edges 3r + j, in the same order
  if (c.a1.vhe) {
    const int h0 = c.a.vhe[v];
    c.a1.vhe[v] = 4 * h0 - h0 % 3;
  }
}

template <int BLK>
__global__ void __launch_bounds__(BLK) k_loop_face(TriStep c) {
  // the 12-int rows of every face (children, and when carried their twins
  // and edge ids) are contiguous over the wave: they leave through LDS
  __shared__ uint32_t stage[BLK / 64][64 * 13];
  const int rid = blockIdx.x * blockDim.x + threadIdx.x;
  const bool valid = rid < c.t.F;
  const int r = valid ? rid : c.t.F - 1;
  const int l = threadIdx.x & 63;
  uint32_t *lds = stage[threadIdx.x >> 6];
  const long long rw = (long long)rid - l;             // first face of the wave
  const int cnt = (int)min(64ll, (long long)c.t.F - rw) * 12;
  const int V = c.t.V;
  const int v0 = c.t.fv[3 * r], v1 = c.t.fv[3 * r + 1], v2 = c.t.fv[3 * r + 2];
  const int e0 = V + c.a.eid[3 * r], e1 = V + c.a.eid[3 * r + 1], e2 = V + c.a.eid[3 * r + 2];
  {
    const uint32_t row[12] = {(uint32_t)v0, (uint32_t)e0, (uint32_t)e2, (uint32_t)v1, (uint32_t)e1, (uint32_t)e0,
                              (uint32_t)v2, (uint32_t)e2, (uint32_t)e1, (uint32_t)e0, (uint32_t)e1, (uint32_t)e2};
    wave_store<12>(lds, row, reinterpret_cast<uint32_t *>(c.fv1) + 12 * rw, l, cnt);
  }
  if (!c.a1.twin) return;
  // ---- carried adjacency of level k+1 (see above); h1(q, s) = 3 q + s
  const int vv[3] = {v0, v1, v2};
  int ed[3], tw[3];
#pragma unroll
  for (int j = 0; j < 3; ++j) {
    ed[j] = c.a.eid[3 * r + j];
    tw[j] = c.a.twin[3 * r + j];
  }
  uint32_t tw1[12], ei1[12];
  const int q3 = 4 * r + 3;
#pragma unroll
  for (int j = 0; j < 3; ++j) {
    const int jn = (j + 1) % 3, jp = (j + 2) % 3;
    const int t = tw[j], tp = tw[jp];
    // child j = (v_j, E_j, E_{j-1}): v_j -> E_j is the first half of 3r+j; its
    // twin E_j -> v_j is the last slot of the child of the face across e_j at v_j
    tw1[3 * j + 0] = t < 0 ? -1 : 3 * (4 * (t / 3) + (t % 3 + 1) % 3) + 2;
    tw1[3 * j + 1] = 3 * q3 + jp;                                           // E_j -> E_{j-1}
    tw1[3 * j + 2] = tp < 0 ? -1 : 3 * (4 * (tp / 3) + tp % 3);           // E_{j-1} -> v_j
    tw1[9 + j] = 3 * (4 * r + jn) + 1;                                      // centre: E_j -> E_{j+1}
    ei1[3 * j + 0] = c.base[ed[j]] + (vv[j] > vv[jn]);
    ei1[3 * j + 2] = c.base[ed[jp]] + (vv[j] > vv[jp]);
  }
#pragma unroll
  for (int m = 0; m < 3; ++m) {
    // centre edge (E_{e_m}, E_{e_{m+1}}): child 3 slot m and child m+1 slot 1
    const int mn = (m + 1) % 3, mo = (m + 2) % 3;
    const int a = min(ed[m], ed[mn]), b = max(ed[m], ed[mn]), other = ed[mo];
    const int hb = 3 * r + (ed[m] == b ? m : mn);  // b's half-edge in face r
    const int tb = c.a.twin[hb];
    int rank = 2 + (other < a);
    if (tb >= 0) {
      rank += lt_new(c.a.eid[he_next<3>(c.t, tb)], a, a, other);
      rank += lt_new(c.a.eid[he_prev<3>(c.t, tb)], a, a, other);
    }
    const int id = c.base[b] + rank;
    ei1[9 + m] = id;
    ei1[3 * mn + 1] = id;
    if (valid) c.a1.e2h[id] = 3 * (4 * r + mn) + 1;  // the lower of its two half-edges
  }
  wave_store<12>(lds, tw1, reinterpret_cast<uint32_t *>(c.a1.twin) + 12 * rw, l, cnt);
  wave_store<12>(lds, ei1, reinterpret_cast<uint32_t *>(c.a1.eid) + 12 * rw, l, cnt);
  if (!valid) return;
  // edges owned by this face (its half-edge is the lower of the pair): the
  // halves' owners and the canonical half-edge of the edge point
#pragma unroll
  for (int j = 0; j < 3; ++j) {
    const int t = tw[j], jn = (j + 1) % 3;
    if (t >= 0 && t < 3 * r + j) continue;
    const int b0 = c.base[ed[j]];
    c.a1.e2h[b0 + (vv[j] > vv[jn])] = 3 * (4 * r + j);          // (v_j, E_j): v_j -> E_j
    c.a1.e2h[b0 + (vv[jn] > vv[j])] = 3 * (4 * r + jn) + 2;     // (v_{j+1}, E_j): E_j -> v_{j+1}
    c.a1.vhe[c.t.V + ed[j]] = t < 0 ? 3 * (4 * r + jn) + 2      // boundary: E_j -> v_{j+1} starts the fan
                                    : min(min(3 * (4 * r + j) + 1, 3 * (4 * r + jn) + 2), 3 * q3 + j);
  }
}

// ------------------------------------------------------------------ sqrt(3)
// Carried adjacency of the next level (App. A topology: child 3r+j =
// (v_j, X_j, F_r) with X_j = F_s across an interior edge j, else v_{j+1};
// F_r = |v| + r). The boundary edges (v_j, v_{j+1}) are the only edges of
// level k+1 whose ends are both old vertices, so they come first in the
// (hi, lo) order and keep their relative order: ids 0 .. B-1, i.e. the
// level-k boundary prefix. Every other edge has a face point F_r as its
// higher end; its lower neighbours, ascending, are the three corners of r
// and the face points F_s of the neighbours s < r. With base = exclusive
// scan of 3 + |{neighbours s < r}| over the faces:
//   (v, F_r) -> B + base(r) + rank of v among r's corners,
//   (F_x, F_m), x < m -> B + base(m) + 3 + |{neighbours s of m, s < x}|.
template <int BLK>
__global__ void __launch_bounds__(BLK) k_sqrt3_count(TriStep c) {
  const int r = blockIdx.x * blockDim.x + threadIdx.x;
  if (r >= c.t.F) return;
  int cnt = 3;
#pragma unroll
  for (int j = 0; j < 3; ++j) {
    const int t = c.a.twin[3 * r + j];
    cnt += (t >= 0 && t / 3 < r);
  }
  c.base[r] = cnt;
}

__device__ __forceinline__ int rank3(int x, int a, int b) { return (x > a) + (x > b); }

template <int BLK>
__global__ void __launch_bounds__(BLK) k_sqrt3_face(TriStep c) {
  // the 9-int rows of every face (children, and when carried their twins and
  // edge ids) are contiguous over the wave: they leave through LDS
  __shared__ uint32_t stage[BLK / 64][64 * 9];
  const int rid = blockIdx.x * blockDim.x + threadIdx.x;
  const bool valid = rid < c.t.F;
  const int r = valid ? rid : c.t.F - 1;
  const int l = threadIdx.x & 63;
  uint32_t *lds = stage[threadIdx.x >> 6];
  const long long rw = (long long)rid - l;  // first face of the wave
  const int cnt = (int)min(64ll, (long long)c.t.F - rw) * 9;
  const int V = c.t.V;
  int v[3], tw[3];
#pragma unroll
  for (int j = 0; j < 3; ++j) {
    v[j] = c.t.fv[3 * r + j];
    tw[j] = c.a.twin[3 * r + j];
  }
  if (valid) {
    const f3 sum = add3(add3(ld3(c.P, v[0]), ld3(c.P, v[1])), ld3(c.P, v[2]));
    st3(c.P1, V + r, mul3(1.0f / 3.0f, sum));
  }
  if (c.fv1) {  // (before the last step from level k, only the caller wants it)
    uint32_t row[9];
#pragma unroll
    for (int j = 0; j < 3; ++j) {
      row[3 * j + 0] = v[j];
      row[3 * j + 1] = tw[j] < 0 ? v[(j + 1) % 3] : V + tw[j] / 3;
      row[3 * j + 2] = V + r;
    }
    wave_store<9>(lds, row, reinterpret_cast<uint32_t *>(c.fv1) + 9 * rw, l, cnt);
  }
  if (!c.a1.twin) return;
  // ---- carried adjacency of level k+1 (see above); h1(q, s) = 3 q + s
  // (without c.a1.eid only the twins and ring starts: no edge ids, no face bases)
  const bool ids = c.a1.eid != nullptr;
  const int B = c.nbnd, br = ids ? B + c.base[r] : 0;
  int nb[3];  // neighbour across edge j, -1 on the boundary
#pragma unroll
  for (int j = 0; j < 3; ++j) nb[j] = tw[j] < 0 ? -1 : tw[j] / 3;
  uint32_t tw1[9], ei1[9];
  int vhe_fp = 9 * r + 2;  // F_r -> v_0; F_r is never on the boundary
#pragma unroll
  for (int j = 0; j < 3; ++j) {
    const int jn = (j + 1) % 3, jp = (j + 2) % 3;
    const int t = tw[j], tp = tw[jp];
    const int rk_j = rank3(v[j], v[jn], v[jp]), rk_jn = rank3(v[jn], v[j], v[jp]);
    // slot 2: F_r -> v_j; its twin v_j -> F_r is slot 1 of child j-1 (boundary
    // edge j-1) or slot 0 of the child at v_j of the face across edge j-1
    const int t2 = tp < 0 ? 9 * r + 3 * jp + 1 : 9 * (tp / 3) + 3 * (tp % 3);
    tw1[3 * j + 2] = t2;
    const int id2 = br + rk_j;
    ei1[3 * j + 2] = id2;
    if (ids && valid) c.a1.e2h[id2] = min(9 * r + 3 * j + 2, t2);
    if (t < 0) {
      // boundary edge j kept: v_j -> v_{j+1}, then v_{j+1} -> F_r
      tw1[3 * j + 0] = -1;
      tw1[3 * j + 1] = 9 * r + 3 * jn + 2;
      ei1[3 * j + 1] = br + rk_jn;
      ei1[3 * j + 0] = 0;
      if (ids) {
        const int e = c.a.eid[3 * r + j];
        const int idb = c.a.bscan ? c.a.bscan[e] : e;  // its rank among the boundary edges
        ei1[3 * j + 0] = idb;
        if (valid) c.a1.e2h[idb] = 9 * r + 3 * j;
      }
    } else {
      const int s = t / 3, i = t % 3;  // t = s's half-edge v_{j+1} -> v_j
      // slot 0: v_j -> F_s; twin F_s -> v_j is slot 2 of s's child at v_j
      tw1[3 * j + 0] = 9 * s + 3 * ((i + 1) % 3) + 2;
      // slot 1: F_s -> F_r, the flipped edge; twin F_r -> F_s is slot 1 of s's child i
      tw1[3 * j + 1] = 9 * s + 3 * i + 1;
      if (s < r) vhe_fp = min(vhe_fp, 9 * s + 3 * i + 1);
      ei1[3 * j + 0] = ei1[3 * j + 1] = 0;
      if (ids) {
        const int w = c.t.fv[3 * s + (i + 2) % 3];  // the third corner of s
        ei1[3 * j + 0] = B + c.base[s] + rank3(v[j], v[jn], w);
        int idf;
        if (s < r) {
          idf = br + 3 + (nb[0] >= 0 && nb[0] < s) + (nb[1] >= 0 && nb[1] < s) + (nb[2] >= 0 && nb[2] < s);
        } else {
          int k3 = 0;
#pragma unroll
          for (int m = 0; m < 3; ++m) {
            const int u = c.a.twin[3 * s + m];
            k3 += (u >= 0 && u / 3 < r);
          }
          idf = B + c.base[s] + 3 + k3;
          if (valid) c.a1.e2h[idf] = 9 * r + 3 * j + 1;  // the lower of its two half-edges
        }
        ei1[3 * j + 1] = idf;
      }
    }
  }
  wave_store<9>(lds, tw1, reinterpret_cast<uint32_t *>(c.a1.twin) + 9 * rw, l, cnt);
  if (ids) wave_store<9>(lds, ei1, reinterpret_cast<uint32_t *>(c.a1.eid) + 9 * rw, l, cnt);
  if (valid) c.a1.vhe[V + r] = vhe_fp;
}

template <int BLK>
__global__ void __launch_bounds__(BLK) k_sqrt3_vertex(TriStep c) {
  const int v = blockIdx.x * blockDim.x + threadIdx.x;
  if (v >= c.t.V) return;
  if (c.Vg > 0 && v >= c.Vg) {
    // face point F_r of the previous level: never on the boundary; its ring is
    // r's corners and the face points across r's interior edges, all in the
    // rows of r's three children (v_j, X_j, F_r)
    const int r = v - c.Vg;
    const int32_t *rw = c.t.fv + 9ll * r;
    const f3 p = ld3(c.P, v);
    f3 sum = add3(add3(ld3(c.P, rw[0]), ld3(c.P, rw[3])), ld3(c.P, rw[6]));
    int n = 3;
#pragma unroll
    for (int j = 0; j < 3; ++j) {
      const int x = rw[3 * j + 1];
      if (x >= c.Vg) {
        sum = add3(sum, ld3(c.P, x));
        ++n;
      }
    }
    st3(c.P1, v, sqrt3_pt(p, sum, n));
    if (c.a1.vhe) c.a1.vhe[v] = 3 * c.a.vhe[v];
    return;
  }
  if (c.fp_done && v >= c.Vq && v < c.Vg) {
    // written by the step before, with the closed-form ring of a face point
    // whose three edges are interior (slot 1 of each child pairs with slot 1)
    const int *tr = c.ap.twin + 9ll * (v - c.Vq);
    if (tr[1] % 3 == 1 && tr[4] % 3 == 1 && tr[7] % 3 == 1) return;
  }
  const f3 p = ld3(c.P, v);
  Ring R{{0.f, 0.f, 0.f}, 0, 0, -1};
  if (c.a0.twin && ring_cage_sqrt3(c, v, R)) {
  } else if (c.Vg == 0) {
    if (c.pbslot && v < c.fpV && ring_trisected_old(c, v, R)) {
    } else if (!(v >= c.fpV && v < c.fpV + c.fpF && ring_rows_fp(c.t, c.a, c.P, v, v - c.fpV, R))) {
      R = ring3(c.t, c.a, c.P, v);
    }
  } else {
    R = (c.app.twin && v < c.Vq) ? ring_prev2_sqrt3(c, v) : ring_prev_sqrt3(c, v);
  }
  const f3 S = R.ub >= 0 ? p : sqrt3_pt(p, R.sum, R.faces);
  st3(c.P1, v, S);
  // an old vertex's half-edges at level k+1 are the first slots 3 (3r + j) of
  // the children at its level-k half-edges 3r + j, in the same order
  if (c.a1.vhe) c.a1.vhe[v] = 3 * c.a.vhe[v];
}

// ------------------------------------------------------------ Loop creases
// The paper gives crease rules for Catmull-Clark (Sec. 3.3); Loop takes the
// same rules on its own points: a crease edge's point blends Loop's edge
// point with the midpoint (above); a vertex with k >= 2 incident crease
// edges takes the crease rule 3/4 p + 1/8 (its two crease neighbours)
// (k = 2) or stays (k >= 3), blended with its smooth point by the mean
// sharpness when that is below 1 (boundary vertices keep the boundary rule);
// the two halves of a crease edge inherit sharpness by the Chaikin rule.
__device__ __forceinline__ double chaikin_tri(double si, double sj) {
#pragma clang fp contract(off)
  const double t = 0.25 * (si + 3.0 * sj) - 1.0;  // this operation order, no fused multiply-add
  return t > 0.0 ? t : 0.0;
}

// Per level-k vertex, after the smooth vertex points: crease valency and the
// first two incident creases (kept for the inheritance), then the crease or
// corner rule over the smooth point. The walk visits every incident edge
// (the outgoing half-edges, and the incoming boundary one).
__global__ void __launch_bounds__(kBlock) k_loop_crease_vertex(TriStep c) {
  const int v = blockIdx.x * blockDim.x + threadIdx.x;
  if (v >= c.t.V) return;
  const Adj &a = c.a;
  int k = 0, cv0 = -1, cv1 = -1, ce0 = -1, ce1 = -1;
  double ssum = 0.0;
  auto crease = [&](int e, int w) {
    const double sg = a.sig[e];
    const bool on = sg > 0.0;
    cv0 = (on && k == 0) ? w : cv0;
    ce0 = (on && k == 0) ? e : ce0;
    cv1 = (on && k == 1) ? w : cv1;
    ce1 = (on && k == 1) ? e : ce1;
    k += on;
    ssum += on ? sg : 0.0;
  };
  const int h0 = a.vhe[v];
  int h = h0, n = 0;
  bool bnd = false;
  while (true) {
    crease(a.eid[h], c.t.fv[he_next<3>(c.t, h)]);
    ++n;
    const int hp = he_prev<3>(c.t, h);
    const int tw = a.twin[hp];
    if (tw < 0) {  // the incoming boundary half-edge u -> v ends the fan
      bnd = true;
      crease(a.eid[hp], c.t.fv[hp]);
      break;
    }
    if (tw == h0 || n >= SUBDIV_MAX_VALENCE) break;
    h = tw;
  }
  a.vcr[v] = make_int4(k, ce0, ce1, 0);
  if (bnd || k < 2) return;
  const f3 p = ld3(c.P, v);
  const f3 sharp = k == 2 ? loop_bnd_pt(p, add3(ld3(c.P, cv0), ld3(c.P, cv1))) : p;
  const double sm = ssum / (double)k;
  if (sm >= 1.0) {
    st3(c.P1, v, sharp);
  } else {
    const float w = (float)sm;
    st3(c.P1, v, lin2(1.0f - w, ld3(c.P1, v), w, sharp));
  }
}

// Per level-k crease edge e = (lo, hi): its children (lo, E_e) and (hi, E_e)
// are the level-(k+1) edges base(e) and base(e) + 1; each end takes
// sigma_i = the other crease's sharpness when the end has exactly two
// creases, else e's own. The caller has cleared sig1.
__global__ void __launch_bounds__(kBlock) k_loop_crease_edge(TriStep c, double *sig1) {
  const int e = blockIdx.x * blockDim.x + threadIdx.x;
  if (e >= c.a.E) return;
  const double sg = c.a.sig[e];
  if (!(sg > 0.0)) return;
  const int h = c.a.e2h[e];
  const int x = c.t.fv[h], y = c.t.fv[he_next<3>(c.t, h)];
  const int b = c.base[e];
#pragma unroll
  for (int end = 0; end < 2; ++end) {
    const int v = end ? max(x, y) : min(x, y);
    const int4 q = c.a.vcr[v];
    const double si = q.x == 2 ? c.a.sig[q.y == e ? q.z : q.y] : sg;
    sig1[b + end] = chaikin_tri(si, sg);
  }
}

hipError_t loop_crease_launch(const TriStep &c, double *sig1, hipStream_t s) {
  hipLaunchKernelGGL(k_loop_crease_vertex, dim3(grid_for(c.t.V)), dim3(kBlock), 0, s, c);
  if (sig1) hipLaunchKernelGGL(k_loop_crease_edge, dim3(grid_for(c.a.E)), dim3(kBlock), 0, s, c, sig1);
  return hipGetLastError();
}

// ------------------------------------- sqrt(3) with Kobbelt's boundary cycle
// App. A leaves the sqrt(3) boundary to Kobbelt's sqrt(3) work, whose boundary
// rule runs over two steps: the first is the sqrt(3) step with the boundary
// fixed (the kernels above); the second, the trisection step here, splits
// every boundary edge in three. Reading (the oracle's): a face has at most one
// boundary edge (every face after a sqrt(3) step does); a boundary face r with
// boundary edge j = (u, w) gets no face point but two points on that edge, p
// near u at |v| + r (the face point's index) and q near w at |v| + |f| + (rank
// of r among the boundary faces), which stand in for the face point wherever
// a neighbour's flipped edge reaches r: q across r's edge j+1, p across edge
// j+2. Its children are 3r+j = (p, q, v_j+2), 3r+j+1 = (v_j+1, X_j+1, q) and
// 3r+j+2 = (v_j+2, X_j+2, p); interior faces split as in the sqrt(3) step.
// Boundary points follow the ternary refinement of a uniform cubic B-spline
// curve on the boundary polygon (mask [1 4 10 16 19 16 10 4 1] / 27):
// p = (u- + 16 u + 10 w) / 27, q = (10 u + 16 w + w+) / 27, a boundary vertex
// (4 a + 19 v + 4 b) / 27 over its boundary neighbours a, b. Interior vertices
// and face points are those of the sqrt(3) step.

// per face: the slot of its boundary edge (or -1) and a boundary flag (scanned
// into the ranks afterwards); per boundary edge u -> w: w is u's next and u is
// w's previous boundary neighbour
__global__ void __launch_bounds__(kBlock) k_trisect_mark(TrisectStep c) {
  const int r = blockIdx.x * blockDim.x + threadIdx.x;
  if (r >= c.t.F) return;
  int slot = -1;
#pragma unroll
  for (int j = 0; j < 3; ++j)
    if (c.a.twin[3 * r + j] < 0) slot = j;
  c.bslot[r] = slot;
  c.brank[r] = slot >= 0;
  if (slot >= 0) {
    const int u = c.t.fv[3 * r + slot], w = c.t.fv[3 * r + (slot + 1) % 3];
    c.bnb[2 * u + 1] = w;
    c.bnb[2 * w] = u;
  }
}

__global__ void __launch_bounds__(kBlock) k_trisect_vertex(TrisectStep c) {
  const int v = blockIdx.x * blockDim.x + threadIdx.x;
  if (v >= c.t.V) return;
  const f3 p = ld3(c.P, v);
  const int h0 = c.a.vhe[v];
  const bool bnd = c.a.twin[h0] < 0;  // the canonical half-edge of a boundary vertex is its boundary one
  f3 S;
  if (bnd) {
    const f3 nb = add3(ld3(c.P, c.bnb[2 * v]), ld3(c.P, c.bnb[2 * v + 1]));
    S = lin2(19.0f / 27.0f, p, 4.0f / 27.0f, nb);
  } else {
    Ring R{{0.f, 0.f, 0.f}, 0, 0, -1};
    if (c.ap.twin && v < c.fpV) {
      walk_below_sqrt3(c.ap, c.P, c.fpV, c.ap.vhe[v], R);  // level k came from a sqrt(3) step
    } else if (!(v >= c.fpV && v < c.fpV + c.fpF && ring_rows_fp(c.t, c.a, c.P, v, v - c.fpV, R))) {
      R = ring3(c.t, c.a, c.P, v);
    }
    S = sqrt3_pt(p, R.sum, R.faces);
  }
  st3(c.P1, v, S);
  if (c.a1.twin) {
    // start half-edge on level k+1 (see the carried adjacency below): a
    // boundary vertex u leaves along u -> p of the face r whose boundary edge
    // starts at u, which lies in the child at u of the face across r's edge
    // after next; an interior vertex keeps the first slot of the child at its
    // level-k start (the face kernel then lowers it where v is the apex of a
    // boundary face)
    if (bnd) {
      const int t = c.a.twin[3 * (h0 / 3) + (h0 % 3 + 2) % 3];
      c.a1.vhe[v] = 9 * (t / 3) + 3 * (t % 3);
    } else {
      c.a1.vhe[v] = 3 * h0;
    }
  }
}

// Edge counts of level k+1 per higher end: the points V + r (face point, or p
// of a boundary face) come first in id order, then the q points V + F + rank;
// the counts of both runs are scanned together, so base[r] and base[F + rank
// ... ] follow. pmask records which of the face's edges see a V + s point of
// the face across (rather than its q).
__global__ void __launch_bounds__(kBlock) k_trisect_count(TrisectStep c) {
  const int r = blockIdx.x * blockDim.x + threadIdx.x;
  if (r >= c.t.F) return;
  const int F = c.t.F, j = c.bslot[r];
  int s[3];
  bool isp[3];
#pragma unroll
  for (int i = 0; i < 3; ++i) {
    const int t = c.a.twin[3 * r + i];
    s[i] = t < 0 ? -1 : t / 3;
    const int js = t < 0 ? -1 : c.bslot[s[i]];
    isp[i] = t >= 0 && !(js >= 0 && t % 3 == (js + 1) % 3);
  }
  int cp, cq = 0;
  if (j < 0) {
    cp = 3 + (isp[0] && s[0] < r) + (isp[1] && s[1] < r) + (isp[2] && s[2] < r);
  } else {
    const int jn = (j + 1) % 3, jp = (j + 2) % 3;
    cp = 2 + (isp[jp] && s[jp] < r);
    cq = 3 + (isp[jn] || s[jn] < r);
  }
  c.base[r] = cp;
  c.base[F + r] = cq;
  c.pmask[r] = (uint8_t)(isp[0] | (isp[1] << 1) | (isp[2] << 2));
}

// Carried adjacency of level k+1 (h' = 9 r + 3 i + slot; slot s runs from
// corner s to corner s+1 of child 3r+i). Write (s_i, i'_i) for the face across
// edge i of r and the slot of the shared edge in it, so that s's corner i' is
// r's v_{i+1} and its corner i'+1 is r's v_i; X_i is s's point toward r.
// Twins:
//   slot 1 of a child at an interior edge i (X_i -> V + r or -> q): slot 1 of
//     s's child i';
//   v_i -> X_i (slot 0): X_i -> v_i is slot 2 of s's child i'+1 when s has no
//     boundary edge, slot 1 of s's child j_s (q -> its apex) when X_i is s's
//     q, and none when X_i is s's p (then v_i -> p is a boundary segment);
//   V + r -> v_i of an interior face: slot 0 of the child at v_i of the face
//     across edge i-1 (s's child i'');
//   boundary face (j; u, w, z the corners j, j+1, j+2): p -> q and q -> w are
//     boundary segments, q -> z pairs with slot 0 of the child i' of the face
//     across edge j+1, and z -> p (child j) with p -> z (child j+2).
// Edge ids ((hi, lo) order): no edge joins two old vertices, so the runs of
// the points V + r come first (lower neighbours: r's corners, or z and u, then
// the points V + s < V + r of the faces across), then the runs of the q
// points (lower neighbours z and w, then p and a V + s point across edge j+1,
// then an earlier q across it). Boundary edges keep their ranks: u - p of the
// boundary faces in face order, then per boundary face q - w and p - q.
__device__ __forceinline__ void trisect_carry(const TrisectStep &c, int r, bool valid, const int (&v)[3],
                                              const int (&X)[3], uint32_t *lds, long long rw, int l, int cnt) {
  const int V = c.t.V, F = c.t.F, j = c.bslot[r];
  // (without c.a1.eid only the twins and ring starts: no edge ids, no bases)
  const bool ids = c.a1.eid != nullptr;
  const int32_t *baseP = c.base, *baseQ = ids ? c.base + F : nullptr;
  int s[3], ip[3], js[3];
  bool isp[3];
#pragma unroll
  for (int i = 0; i < 3; ++i) {
    const int t = c.a.twin[3 * r + i];
    s[i] = t < 0 ? r : t / 3;  // (a boundary edge's entries are never used)
    ip[i] = t < 0 ? 0 : t % 3;
    js[i] = t < 0 ? -1 : c.bslot[s[i]];
    isp[i] = X[i] >= 0 && X[i] < V + F;
  }
  const int bP = ids ? baseP[r] : 0;
  // edge (v_i, X_i), edge i interior
  auto id_vX = [&](int i, int vi, int vn) {
    if (!isp[i]) return baseQ[s[i]] + (vi > vn);
    if (js[i] >= 0) return baseP[s[i]] + (vi > vn);
    const int w = c.t.fv[3 * s[i] + (ip[i] + 2) % 3];
    return baseP[s[i]] + rank3(vi, vn, w);
  };
  // edge (X_i, V + r), edge i interior; r's own lower V + s neighbours: those
  // across its three edges (no boundary edge), or across edge j+2 alone
  auto id_XP = [&](int i, bool own_bnd) {
    const int x = s[i];
    if (!isp[i]) return baseQ[x] + 2 + (r > x);
    if (x < r) {
      if (own_bnd) return bP + 2;
      return bP + 3 + (isp[0] && s[0] < x) + (isp[1] && s[1] < x) + (isp[2] && s[2] < x);
    }
    if (js[i] >= 0) return baseP[x] + 2;  // the only lower V + s neighbour of x's p is V + r
    int k = 0;
    const uint8_t pm = c.pmask[x];
#pragma unroll
    for (int m = 0; m < 3; ++m) k += ((pm >> m) & 1) && c.a.twin[3 * x + m] / 3 < r;
    return baseP[x] + 3 + k;
  };
  // v_i -> X_i: its twin in the face across (see above)
  auto flip = [&](int i) {
    return js[i] < 0 ? 9 * s[i] + 3 * ((ip[i] + 1) % 3) + 2 : ip[i] == (js[i] + 1) % 3 ? 9 * s[i] + 3 * js[i] + 1 : -1;
  };
  uint32_t tw1[9], ei1[9];
  if (j < 0) {
#pragma unroll
    for (int i = 0; i < 3; ++i) {
      const int in = (i + 1) % 3, im = (i + 2) % 3;
      tw1[3 * i + 0] = flip(i);
      tw1[3 * i + 1] = 9 * s[i] + 3 * ip[i] + 1;
      tw1[3 * i + 2] = 9 * s[im] + 3 * ip[im];
      ei1[3 * i + 0] = ids ? id_vX(i, v[i], v[in]) : 0;
      ei1[3 * i + 1] = ids ? id_XP(i, false) : 0;
      ei1[3 * i + 2] = bP + rank3(v[i], v[in], v[im]);
    }
    if (valid) {
      int m0 = 9 * r + 2;
#pragma unroll
      for (int i = 0; i < 3; ++i) m0 = min(m0, (int)tw1[3 * i + 1]);
      c.a1.vhe[V + r] = m0;
    }
  } else {
    const int bQ = ids ? baseQ[r] : 0;
    int idPQ = 0, idwQ = 0, iduP = 0;
#pragma unroll
    for (int i = 0; i < 3; ++i) {
      const int in = (i + 1) % 3, im = (i + 2) % 3;
      if (i == j) {  // (p, q, z): p -> q, q -> z, z -> p; u = v_i, w = v_in, z = v_im
        idPQ = bQ + 2 + (isp[in] && s[in] < r);
        iduP = bP + (v[i] > v[im]);
        tw1[3 * i + 0] = -1;
        tw1[3 * i + 1] = 9 * s[in] + 3 * ip[in];
        tw1[3 * i + 2] = 9 * r + 3 * im + 2;
        ei1[3 * i + 0] = idPQ;
        ei1[3 * i + 1] = bQ + (v[im] > v[in]);
        ei1[3 * i + 2] = bP + (v[im] > v[i]);
      } else if (i == (j + 1) % 3) {  // (w, X, q): w = v_i, z = v_in
        idwQ = bQ + (v[i] > v[in]);
        tw1[3 * i + 0] = flip(i);
        tw1[3 * i + 1] = 9 * s[i] + 3 * ip[i] + 1;
        tw1[3 * i + 2] = -1;
        ei1[3 * i + 0] = ids ? id_vX(i, v[i], v[in]) : 0;
        ei1[3 * i + 1] = isp[i] ? bQ + 2 + (s[i] > r) : (s[i] < r || !ids ? bQ + 3 : baseQ[s[i]] + 3);
        ei1[3 * i + 2] = idwQ;
      } else {  // (z, X, p): z = v_i, u = v_in
        tw1[3 * i + 0] = flip(i);
        tw1[3 * i + 1] = 9 * s[i] + 3 * ip[i] + 1;
        tw1[3 * i + 2] = 9 * r + 3 * in + 2;
        ei1[3 * i + 0] = ids ? id_vX(i, v[i], v[in]) : 0;
        ei1[3 * i + 1] = ids ? id_XP(i, true) : 0;
        ei1[3 * i + 2] = bP + (v[i] > v[in]);
      }
    }
    if (valid) {
      const int rk = c.brank[r], B = c.nbnd, jn = (j + 1) % 3;
      if (ids) {
        c.a1.bscan[iduP] = rk;  // u - p
        c.a1.bscan[idwQ] = B + 2 * rk;  // q - w
        c.a1.bscan[idPQ] = B + 2 * rk + 1;
      }
      c.a1.vhe[V + r] = 9 * r + 3 * j;
      c.a1.vhe[V + F + rk] = 9 * r + 3 * jn + 2;
      const int z = c.t.fv[3 * r + (j + 2) % 3];
      if (c.a.twin[c.a.vhe[z]] >= 0) atomicMin(&c.a1.vhe[z], 9 * r + 3 * j + 2);  // the apex z -> p
    }
  }
  if (valid && ids) {
    // every edge once, by its lower half-edge (the only one on the boundary)
#pragma unroll
    for (int i = 0; i < 9; ++i) {
      const int h = 9 * r + i, t = (int)tw1[i];
      if (t < 0 || h < t) c.a1.e2h[ei1[i]] = h;
    }
  }
  wave_store<9>(lds, tw1, reinterpret_cast<uint32_t *>(c.a1.twin) + 9 * rw, l, cnt);
  if (ids) wave_store<9>(lds, ei1, reinterpret_cast<uint32_t *>(c.a1.eid) + 9 * rw, l, cnt);
}

__global__ void __launch_bounds__(kBlock) k_trisect_face(TrisectStep c) {
  __shared__ uint32_t stage[kBlock / 64][64 * 9];
  const int rid = blockIdx.x * blockDim.x + threadIdx.x;
  const bool valid = rid < c.t.F;
  const int r = valid ? rid : c.t.F - 1;
  const int l = threadIdx.x & 63;
  uint32_t *lds = stage[threadIdx.x >> 6];
  const long long rw = (long long)rid - l;  // first face of the wave
  const int cnt = (int)min(64ll, (long long)c.t.F - rw) * 9;
  const int V = c.t.V, F = c.t.F;
  int v[3], X[3];
#pragma unroll
  for (int i = 0; i < 3; ++i) {
    v[i] = c.t.fv[3 * r + i];
    const int t = c.a.twin[3 * r + i];
    X[i] = -1;
    if (t >= 0) {  // the neighbour's point toward r: its face point, or its q across its edge after the boundary one
      const int s = t / 3, js = c.bslot[s];
      X[i] = (js >= 0 && t % 3 == (js + 1) % 3) ? V + F + c.brank[s] : V + s;
    }
  }
  const int j = c.bslot[r];
  const int P_ = V + r, Q = j >= 0 ? V + F + c.brank[r] : -1;
  if (valid) {
    if (j < 0) {
      const f3 sum = add3(add3(ld3(c.P, v[0]), ld3(c.P, v[1])), ld3(c.P, v[2]));
      st3(c.P1, V + r, mul3(1.0f / 3.0f, sum));
    } else {
      const int u = v[j], w = v[(j + 1) % 3];
      const f3 pu = ld3(c.P, u), pw = ld3(c.P, w);
      const f3 pum = ld3(c.P, c.bnb[2 * u]), pwp = ld3(c.P, c.bnb[2 * w + 1]);
      st3(c.P1, P_, add3(lin2(1.0f / 27.0f, pum, 16.0f / 27.0f, pu), mul3(10.0f / 27.0f, pw)));
      st3(c.P1, Q, add3(lin2(10.0f / 27.0f, pu, 16.0f / 27.0f, pw), mul3(1.0f / 27.0f, pwp)));
    }
  }
  uint32_t row[9];
#pragma unroll
  for (int i = 0; i < 3; ++i) {
    int a0 = v[i], a1 = X[i], a2 = V + r;  // interior: (v_i, X_i, F_r)
    if (j >= 0) {
      if (i == j) {
        a0 = P_, a1 = Q, a2 = v[(i + 2) % 3];
      } else if (i == (j + 1) % 3) {
        a2 = Q;
      } else {
        a2 = P_;
      }
    }
    row[3 * i + 0] = a0;
    row[3 * i + 1] = a1;
    row[3 * i + 2] = a2;
  }
  wave_store<9>(lds, row, reinterpret_cast<uint32_t *>(c.fv1) + 9 * rw, l, cnt);
  if (!c.a1.twin) return;
  trisect_carry(c, r, valid, v, X, lds, rw, l, cnt);
}

hipError_t trisect_launch(int which, const TrisectStep &c, hipStream_t s) {
  if (which == TRISECT_MARK)
    hipLaunchKernelGGL(k_trisect_mark, dim3(grid_for(c.t.F)), dim3(kBlock), 0, s, c);
  else if (which == TRISECT_FACE)
    hipLaunchKernelGGL(k_trisect_face, dim3(grid_for(c.t.F)), dim3(kBlock), 0, s, c);
  else if (which == TRISECT_COUNT)
    hipLaunchKernelGGL(k_trisect_count, dim3(grid_for(c.t.F)), dim3(kBlock), 0, s, c);
  else
    hipLaunchKernelGGL(k_trisect_vertex, dim3(grid_for(c.t.V)), dim3(kBlock), 0, s, c);
  return hipGetLastError();
}

// ------------------------------------------------------- Loop, last step
// Level k+1 computed from level m = k-1, the level that level k was refined
// from. With E_j = |v_m| + e_j for the edges e_j of a level-m face
// r = (v_0, v_1, v_2):
//   level-k children of r: 4r+j = (v_j, E_j, E_{j-1}), 4r+3 = (E_0, E_1, E_2);
//   level-k edge ids: the carried form of the face kernel above, on level m;
//   level-(k+1) children of a level-k face q = (w_0, w_1, w_2) with edges
//     (x_0, x_1, x_2): 4q+i = (w_i, V_k + x_i, V_k + x_{i-1}),
//     4q+3 = (V_k + x_0, V_k + x_1, V_k + x_2). So r's sixteen grandchildren
//     are the rows 16r .. 16r+15 of level k+1: 48 ints per level-m face.
// Every level-k edge has an edge point E_e as its higher end, and the edges
// with higher end E_e take the ids base(e) .. base(e+1)-1; one lane per
// level-m edge e therefore writes the level-(k+1) edge points of a run of
// ids, and the runs of a wave are contiguous. With e = (a, b) in face r,
// whose other edges are ra (at a) and rb (at b), and in the face s across,
// whose other edges are sa and sb, the level-k edges with higher end E_e and
// their opposite corners are
//   (a, E_e): E_ra and E_sa;          (b, E_e): E_rb and E_sb;
//   (E_ra, E_e): a and E_rb;          (E_rb, E_e): b and E_ra;  likewise in s;
// the vertex point of E_e (valence 6, or a boundary vertex between a and b)
// takes the same points. Sums keep the operand grouping of the per-level
// kernels above (two-term sums commute) and the stencils are the same
// uncontracted ones, so both give the same bits.
template <int BLK>
__global__ void __launch_bounds__(BLK) k_loopl_face(TriLag c) {
  __shared__ int4 stage[BLK / 64][32 * 13];
  const int F = c.tm.F;
  const int rid = blockIdx.x * blockDim.x + threadIdx.x;
  const int r = rid < F ? rid : F - 1;  // every lane takes part in the staged store
  const int l = threadIdx.x & 63;
  int4 *lds = stage[threadIdx.x >> 6];
  const long long rw = (long long)rid - l;                 // first face of the wave
  const int cnt = (int)min(64ll, (long long)F - rw) * 12;  // int4s of the wave's run
  const int Vm = c.tm.V, Vk = c.Vk;
  int v[3], ed[3];
#pragma unroll
  for (int j = 0; j < 3; ++j) {
    v[j] = c.tm.fv[3 * r + j];
    ed[j] = c.am.eid[3 * r + j];
  }
  int xk[12];  // level-k edge ids of the children's half-edges, 3 (q - 4r) + slot
#pragma unroll
  for (int j = 0; j < 3; ++j) {
    const int jn = (j + 1) % 3, jp = (j + 2) % 3;
    xk[3 * j + 0] = c.base[ed[j]] + (v[j] > v[jn]);
    xk[3 * j + 2] = c.base[ed[jp]] + (v[j] > v[jp]);
  }
#pragma unroll
  for (int m = 0; m < 3; ++m) {
    // centre edge (E_{e_m}, E_{e_{m+1}}): child 3 slot m and child m+1 slot 1
    const int mn = (m + 1) % 3, mo = (m + 2) % 3;
    const int a = min(ed[m], ed[mn]), b = max(ed[m], ed[mn]), other = ed[mo];
    const int tb = c.am.twin[3 * r + (ed[m] == b ? m : mn)];
    int rank = 2 + (other < a);
    if (tb >= 0) {
      rank += lt_new(c.am.eid[he_next<3>(c.tm, tb)], a, a, other);
      rank += lt_new(c.am.eid[he_prev<3>(c.tm, tb)], a, a, other);
    }
    xk[9 + m] = xk[3 * mn + 1] = c.base[b] + rank;
  }
  const int E0 = Vm + ed[0], E1 = Vm + ed[1], E2 = Vm + ed[2];
  const int wk[12] = {v[0], E0, E2, v[1], E1, E0, v[2], E2, E1, E0, E1, E2};
  int out[48];
#pragma unroll
  for (int q = 0; q < 4; ++q) {
#pragma unroll
    for (int i = 0; i < 3; ++i) {
      out[12 * q + 3 * i + 0] = wk[3 * q + i];
      out[12 * q + 3 * i + 1] = Vk + xk[3 * q + i];
      out[12 * q + 3 * i + 2] = Vk + xk[3 * q + (i + 2) % 3];
      out[12 * q + 9 + i] = Vk + xk[3 * q + i];
    }
  }
  // 12 int4 per lane, leaving through LDS: half the wave's faces at a time
  // (half the LDS, twice the occupancy), 6 instructions of 64 int4 (1 KB
  // contiguous) per half
#pragma unroll
  for (int hf = 0; hf < 2; ++hf) {
    if ((l >> 5) == hf) {
#pragma unroll
      for (int x = 0; x < 12; ++x)
        lds[13 * (l & 31) + x] = make_int4(out[4 * x], out[4 * x + 1], out[4 * x + 2], out[4 * x + 3]);
    }
    __builtin_amdgcn_wave_barrier();
    int4 *dst = reinterpret_cast<int4 *>(c.fv2) + 12 * (rw + 32 * hf);
#pragma unroll
    for (int t = 0; t < 6; ++t) {
      const int g = 64 * t + l, src = g / 12;
      const int4 x = lds[13 * src + (g - 12 * src)];
      if (g + 384 * hf < cnt) stream_store4(dst + g, x);
    }
    __builtin_amdgcn_wave_barrier();
  }
}

template <int BLK>
__global__ void __launch_bounds__(BLK) k_loopl_edge(TriLag c) {
  __shared__ uint32_t stage[BLK / 64][64 * 18];
  const int E = c.am.E;
  const int eid = blockIdx.x * blockDim.x + threadIdx.x;
  const int e = eid < E ? eid : E - 1;  // every lane takes part in the staged stores
  const int l = threadIdx.x & 63;
  uint32_t *lds = stage[threadIdx.x >> 6];
  const int Vm = c.tm.V, Vk = c.Vk;
  const int h = c.am.e2h[e], r = h / 3, j = h - 3 * r;
  const int jn = j == 2 ? 0 : j + 1, jp = j == 0 ? 2 : j - 1;
  const int a = c.tm.fv[h], b = c.tm.fv[3 * r + jn];
  const int ra = c.am.eid[3 * r + jp], rb = c.am.eid[3 * r + jn];
  const int t = c.am.twin[h];
  const f3 pa = ld3(c.Pk, a), pb = ld3(c.Pk, b), pE = ld3(c.Pk, Vm + e);
  const f3 pra = ld3(c.Pk, Vm + ra), prb = ld3(c.Pk, Vm + rb);
  const int base = c.base[e];
  const int base0 = __shfl(base, 0, 64);
  const int off = 3 * (base - base0);
  auto put = [&](int slot, f3 p) {
    lds[off + 3 * slot + 0] = __float_as_uint(p.x);
    lds[off + 3 * slot + 1] = __float_as_uint(p.y);
    lds[off + 3 * slot + 2] = __float_as_uint(p.z);
  };
  const int lo_slot = a < b ? 0 : 1;  // (a, E_e) is base + 0 when a is the lower old end
  int sa_ = INT_MAX, sb_ = INT_MAX;  // s's edges at a and b (none on the boundary)
  f3 S, S2{0.f, 0.f, 0.f};
  int n;
  if (t < 0) {
    S = loop_bnd_pt(pE, add3(pa, pb));
    const f3 ha = mul3(0.5f, add3(pa, pE)), hb = mul3(0.5f, add3(pb, pE));
    put(lo_slot, ha);
    put(1 - lo_slot, hb);
    n = 2;
    if (ra < e) put(2 + (rb < ra), loop_edge_pt(add3(pra, pE), add3(pa, prb)));
    if (rb < e) put(2 + (ra < rb), loop_edge_pt(add3(prb, pE), add3(pb, pra)));
    n += (ra < e) + (rb < e);
    // two levels up, E_e stays on the boundary between the halves' edge points
    if (c.Pk2) S2 = loop_bnd_pt(S, add3(ha, hb));
  } else {
    const int s = t / 3, i = t - 3 * s;  // t = s's half-edge b -> a
    const int sa = c.am.eid[3 * s + (i == 2 ? 0 : i + 1)], sb = c.am.eid[3 * s + (i == 0 ? 2 : i - 1)];
    sa_ = sa;
    sb_ = sb;
    const f3 psa = ld3(c.Pk, Vm + sa), psb = ld3(c.Pk, Vm + sb);
    S = loop_v6_pt(pE, add3(add3(pa, pb), add3(add3(pra, prb), add3(psa, psb))));
    const f3 ea = loop_edge_pt(add3(pa, pE), add3(pra, psa)), eb = loop_edge_pt(add3(pb, pE), add3(prb, psb));
    put(lo_slot, ea);
    put(1 - lo_slot, eb);
    // the edges (E_x, E_e), x in N(e) = {ra, rb, sa, sb}: their ends and the
    // two corners across them (the end x shares with e, and E of the face's
    // third edge), grouped as the lane of max(x, e) groups them
    const f3 mra = loop_edge_pt(add3(pra, pE), add3(pa, prb)), mrb = loop_edge_pt(add3(prb, pE), add3(pb, pra));
    const f3 msa = loop_edge_pt(add3(psa, pE), add3(pa, psb)), msb = loop_edge_pt(add3(psb, pE), add3(pb, psa));
    // the lower neighbours E_x, x < e, ranked among N(e)
    auto rank = [&](int x) { return (ra < x) + (rb < x) + (sa < x) + (sb < x); };
    if (ra < e) put(2 + rank(ra), mra);
    if (rb < e) put(2 + rank(rb), mrb);
    if (sa < e) put(2 + rank(sa), msa);
    if (sb < e) put(2 + rank(sb), msb);
    n = 2 + (ra < e) + (rb < e) + (sa < e) + (sb < e);
    if (c.Pk2) {
      // E_e's level-(k+1) ring, the six points above, in the order of the
      // old-vertex walk from its level-k start h0. h0 is slot 1 of the corner
      // child at e's first end in one of e's faces (taking e in that face's
      // direction): the ring then runs E of the face's edge before e, the
      // first end, E of the other face's edges at the first end and at the
      // second, the second end, E of the face's edge after e. Or h0 is slot 2
      // of the corner child at the second end: the same cycle from the fifth.
      const int h0 = c.vhek[Vm + e];
      const bool rs = h0 / 12 == r, first = h0 % 3 == 1;
      const f3 w[6] = {sel3(rs, mra, msb), sel3(rs, ea, eb),  sel3(rs, msa, mrb),
                       sel3(rs, msb, mra), sel3(rs, eb, ea), sel3(rs, mrb, msa)};
      f3 sum{0.f, 0.f, 0.f};
#pragma unroll
      for (int x = 0; x < 6; ++x) sum = add3(sum, sel3(first, w[x], w[(x + 4) % 6]));
      S2 = loop_old_pt(S, sum, 6);
    }
  }
  if (c.edges && eid < E) {
    // level k's edges with higher end E_e, in id order: (lo, E_e), (hi, E_e),
    // then (E_x, E_e) for x in N(e), x < e, ascending
    int2 *o = reinterpret_cast<int2 *>(c.edges) + base;
    const int hiE = Vm + e;
    o[0] = make_int2(min(a, b), hiE);
    o[1] = make_int2(max(a, b), hiE);
    int x[4] = {ra, rb, t < 0 ? INT_MAX : c.am.eid[3 * (t / 3) + ((t % 3) == 2 ? 0 : (t % 3) + 1)],
                t < 0 ? INT_MAX : c.am.eid[3 * (t / 3) + ((t % 3) == 0 ? 2 : (t % 3) - 1)]};
#pragma unroll
    for (int i = 0; i < 4; ++i) {
      if (x[i] >= e) continue;
      int rk = 0;
#pragma unroll
      for (int j = 0; j < 4; ++j) rk += (j != i && x[j] < x[i]);
      o[2 + rk] = make_int2(Vm + x[i], hiE);
    }
  }
  __builtin_amdgcn_wave_barrier();
  {
    const int end = min(__shfl(base + n, min(63, E - 1 - (eid - l)), 64), c.Ek);
    const int count = (eid - l < E) ? 3 * (end - base0) : 0;
    uint32_t *dst = reinterpret_cast<uint32_t *>(c.P2 + 3ll * (Vk + base0));
    run_store(lds, dst, count, l);
  }
  __builtin_amdgcn_wave_barrier();
  if (c.cnt1) {
    // level k's own edge counts, 2 + |N below|, over the same run of ids. An
    // end edge (a, E_e) lies in the corner children at a: its other edges
    // there, (E_ra, a) and (a, E_sa), sit in the runs of ra and sa, so they
    // come first exactly when ra < e (sa < e); (E_e, E_ra) and (E_sa, E_e)
    // come after it. An edge (E_x, E_e), x < e, lies in the corner child at
    // the end c shared with x and in the centre child of their face, whose
    // third edge is y: (c, E_e) and (c, E_x) always come first, (E_y, E_e)
    // when y < x, (E_x, E_y) when y < e.
    const int ka = 2 + (ra < e) + (t >= 0 && sa_ < e), kb = 2 + (rb < e) + (t >= 0 && sb_ < e);
    lds[base - base0 + lo_slot] = ka;
    lds[base - base0 + 1 - lo_slot] = kb;
    auto mid = [&](int x, int y, int slot) { lds[base - base0 + slot] = 4 + (y < x) + (y < e); };
    if (t < 0) {
      if (ra < e) mid(ra, rb, 2 + (rb < ra));
      if (rb < e) mid(rb, ra, 2 + (ra < rb));
    } else {
      auto rank = [&](int x) { return (ra < x) + (rb < x) + (sa_ < x) + (sb_ < x); };
      if (ra < e) mid(ra, rb, 2 + rank(ra));
      if (rb < e) mid(rb, ra, 2 + rank(rb));
      if (sa_ < e) mid(sa_, sb_, 2 + rank(sa_));
      if (sb_ < e) mid(sb_, sa_, 2 + rank(sb_));
    }
    __builtin_amdgcn_wave_barrier();
    const int end = min(__shfl(base + n, min(63, E - 1 - (eid - l)), 64), c.Ek);
    const int count = (eid - l < E) ? end - base0 : 0;
    run_store(lds, reinterpret_cast<uint32_t *>(c.cnt1) + base0, count, l);
    __builtin_amdgcn_wave_barrier();
  }
  {
    const uint32_t row[3] = {__float_as_uint(S.x), __float_as_uint(S.y), __float_as_uint(S.z)};
    const int count = 3 * (int)min(64ll, (long long)E - (eid - l));
    wave_store<3>(lds, row, reinterpret_cast<uint32_t *>(c.P2 + 3ll * (Vm + eid - l)), l, count);
    if (c.Pk2) {
      const uint32_t row2[3] = {__float_as_uint(S2.x), __float_as_uint(S2.y), __float_as_uint(S2.z)};
      wave_store<3>(lds, row2, reinterpret_cast<uint32_t *>(c.Pk2 + 3ll * (Vm + eid - l)), l, count);
    }
  }
}

// ----------------------------------------------------- sqrt(3), last step
// Level k+1 from level m = k-1. With twin t_j of the half-edge v_j -> v_{j+1}
// of a level-m face r and X_j = F_s across an interior edge j (t_j = 3s + i),
// else v_{j+1}, level k's child q = 3r + j = (v_j, X_j, F_r) has, across its
//   edge 0 (v_j -> X_j): s's child at v_j, 3s + (i+1) mod 3, or the boundary;
//   edge 1 (X_j -> F_r): s's child i, i.e. face t_j, or r's child j+1 when
//     edge j is on the boundary;
//   edge 2 (F_r -> v_j): face t_{j-1} across edge j-1, or r's child j-1.
// So per level-m face r one lane writes r's nine grandchildren (rows
// 9r .. 9r+8 of level k+1: (w_i, face point across edge i or w_{i+1},
// face point of q)), the face points of r's three children and the vertex
// point of F_r (r's corners and the face points across its interior edges).
// The sums are those of the per-level kernels, in the same order.
template <int BLK>
__global__ void __launch_bounds__(BLK) k_sqrt3l_face(TriLag c) {
  __shared__ uint32_t stage[BLK / 64][64 * 27];
  const int F = c.tm.F;
  const int rid = blockIdx.x * blockDim.x + threadIdx.x;
  const int r = rid < F ? rid : F - 1;  // every lane takes part in the staged stores
  const int l = threadIdx.x & 63;
  uint32_t *lds = stage[threadIdx.x >> 6];
  const long long rw = (long long)rid - l;  // first face of the wave
  const int nw = (int)min(64ll, (long long)F - rw);
  const int Vm = c.tm.V, Vk = c.Vk;
  int v[3], tw[3], X[3];
#pragma unroll
  for (int j = 0; j < 3; ++j) {
    v[j] = c.tm.fv[3 * r + j];
    tw[j] = c.am.twin[3 * r + j];
  }
#pragma unroll
  for (int j = 0; j < 3; ++j) X[j] = tw[j] < 0 ? v[(j + 1) % 3] : Vm + tw[j] / 3;
  const int Fr = Vm + r;
  f3 pv[3], pX[3];
#pragma unroll
  for (int j = 0; j < 3; ++j) pv[j] = ld3(c.Pk, v[j]);
#pragma unroll
  for (int j = 0; j < 3; ++j) pX[j] = tw[j] < 0 ? pv[(j + 1) % 3] : ld3(c.Pk, X[j]);
  const f3 pF = ld3(c.Pk, Fr);
  {
    uint32_t row[27];
#pragma unroll
    for (int j = 0; j < 3; ++j) {
      const int jn = (j + 1) % 3, jp = (j + 2) % 3;
      const int t = tw[j], tp = tw[jp];
      const int q = Vk + 3 * r + j;  // face point of level-k face 3r + j
      const int y0 = t < 0 ? X[j] : Vk + 3 * (t / 3) + (t % 3 + 1) % 3;
      const int y1 = Vk + (t < 0 ? 3 * r + jn : t);
      const int y2 = Vk + (tp < 0 ? 3 * r + jp : tp);
      const int w[3] = {v[j], X[j], Fr}, y[3] = {y0, y1, y2};
#pragma unroll
      for (int i = 0; i < 3; ++i) {
        row[9 * j + 3 * i + 0] = w[i];
        row[9 * j + 3 * i + 1] = y[i];
        row[9 * j + 3 * i + 2] = q;
      }
    }
    if (c.fv2) wave_store<27>(lds, row, reinterpret_cast<uint32_t *>(c.fv2) + 27 * rw, l, 27 * nw);
  }
  {
    uint32_t fp[9];
#pragma unroll
    for (int j = 0; j < 3; ++j) {
      const f3 f = mul3(1.0f / 3.0f, add3(add3(pv[j], pX[j]), pF));
      fp[3 * j + 0] = __float_as_uint(f.x);
      fp[3 * j + 1] = __float_as_uint(f.y);
      fp[3 * j + 2] = __float_as_uint(f.z);
    }
    wave_store<9>(lds, fp, reinterpret_cast<uint32_t *>(c.P2 + 3ll * (Vk + 3 * rw)), l, 9 * nw);
  }
  {
    f3 sum = add3(add3(pv[0], pv[1]), pv[2]);
    int n = 3;
#pragma unroll
    for (int j = 0; j < 3; ++j)
      if (tw[j] >= 0) {
        sum = add3(sum, pX[j]);
        ++n;
      }
    const f3 S = sqrt3_pt(pF, sum, n);
    const uint32_t row[3] = {__float_as_uint(S.x), __float_as_uint(S.y), __float_as_uint(S.z)};
    wave_store<3>(lds, row, reinterpret_cast<uint32_t *>(c.P2 + 3ll * (Vm + rw)), l, 3 * nw);
    if (c.Pk2) {
      // F_r two levels up, when r's three edges are interior (else the old-
      // vertex kernel walks it): its level-(k+1) ring alternates the face
      // points of the level-k faces across F_r -> v_j, the child of the face
      // across edge j-1 at v_j, (v_j, F_r, F_s) in its slot order (formed
      // as that face's lane forms it), and of r's child j; the walk starts at
      // the first of these, or at r's child j when the start h0 is the twin of
      // that child's slot 1, 3 t_j + 1. (Next to the boundary the row gets F_r's
      // level-(k+1) point as a placeholder; the last step's walk replaces it.)
      f3 S2 = S;
      if (tw[0] >= 0 && tw[1] >= 0 && tw[2] >= 0) {
        auto fq = [&](f3 x, f3 y, f3 z) { return mul3(1.0f / 3.0f, add3(add3(x, y), z)); };
        const f3 n0 = fq(pv[0], pF, pX[2]), c0 = fq(pv[0], pX[0], pF);
        const f3 n1 = fq(pv[1], pF, pX[0]), c1 = fq(pv[1], pX[1], pF);
        const f3 n2 = fq(pv[2], pF, pX[1]), c2 = fq(pv[2], pX[2], pF);
        const int h0 = c.vhek[Fr];
        const f3 z{0.f, 0.f, 0.f};
        f3 ring;
        if (h0 == 3 * tw[0] + 1) ring = sum6(z, c0, n1, c1, n2, c2, n0);
        else if (h0 == 3 * tw[1] + 1) ring = sum6(z, c1, n2, c2, n0, c0, n1);
        else if (h0 == 3 * tw[2] + 1) ring = sum6(z, c2, n0, c0, n1, c1, n2);
        else ring = sum6(z, n0, c0, n1, c1, n2, c2);
        S2 = sqrt3_pt(S, ring, 6);
      }
      const uint32_t row2[3] = {__float_as_uint(S2.x), __float_as_uint(S2.y), __float_as_uint(S2.z)};
      wave_store<3>(lds, row2, reinterpret_cast<uint32_t *>(c.Pk2 + 3ll * (Vm + rw)), l, 3 * nw);
    }
  }
  if (c.edges && rid < F) {
    // level k's edge list (the carried ids of the face kernel above): a kept
    // boundary edge j of r keeps its id (the boundary edges of a refined level
    // are its first ids); the edges with higher end F_r take Bk + base(r) +
    // the rank of the lower end among r's corners, then Bk + base(r) + 3 +
    // the rank of F_s among r's neighbours s < r
    int2 *o = reinterpret_cast<int2 *>(c.edges);
    const int br = c.Bk + c.base[r];
    int nb[3];
#pragma unroll
    for (int j = 0; j < 3; ++j) nb[j] = tw[j] < 0 ? INT_MAX : tw[j] / 3;
#pragma unroll
    for (int j = 0; j < 3; ++j) {
      const int jn = (j + 1) % 3, jp = (j + 2) % 3;
      if (tw[j] < 0) {
        const int e = c.am.eid[3 * r + j];
        o[e] = make_int2(min(v[j], v[jn]), max(v[j], v[jn]));
      }
      o[br + (v[j] > v[jn]) + (v[j] > v[jp])] = make_int2(v[j], Fr);
      if (nb[j] < r)
        o[br + 3 + (nb[jn] < nb[j]) + (nb[jp] < nb[j])] = make_int2(Vm + nb[j], Fr);
    }
  }
}

hipError_t tri_lag_launch(int which, const TriLag &c, hipStream_t s) {
  if (which == LAG_LOOP_FACE)
    SUBDIV_LAUNCH_TUNED(TK_LOOPL_FACE, c.tm.F, s, k_loopl_face, c);
  else if (which == LAG_LOOP_EDGE)
    SUBDIV_LAUNCH_TUNED(TK_LOOPL_EDGE, c.am.E, s, k_loopl_edge, c);
  else
    SUBDIV_LAUNCH_TUNED(TK_SQRT3L_FACE, c.tm.F, s, k_sqrt3l_face, c);
  return hipGetLastError();
}

hipError_t tri_launch(int which, const TriStep &c, hipStream_t s) {
  switch (which) {
    case LOOP_EDGE:
      SUBDIV_LAUNCH_TUNED(TK_LOOP_EDGE, c.a.E, s, k_loop_edge, c);
      break;
    case LOOP_VERTEX:
      SUBDIV_LAUNCH_TUNED(TK_LOOP_VERTEX, c.t.V, s, k_loop_vertex, c);
      break;
    case LOOP_FACE:
      SUBDIV_LAUNCH_TUNED(TK_LOOP_FACE, c.t.F, s, k_loop_face, c);
      break;
    case SQRT3_FACE:
      SUBDIV_LAUNCH_TUNED(TK_SQRT3_FACE, c.t.F, s, k_sqrt3_face, c);
      break;
    case SQRT3_COUNT:
      SUBDIV_LAUNCH_TUNED(TK_SQRT3_COUNT, c.t.F, s, k_sqrt3_count, c);
      break;
    default:
      SUBDIV_LAUNCH_TUNED(TK_SQRT3_VERTEX, c.t.V, s, k_sqrt3_vertex, c);
      break;
  }
  return hipGetLastError();
}

}  // namespace subdiv
