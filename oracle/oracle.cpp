// FP64 serial reference ("oracle") for one AlSub refinement step.
//
// TEST INFRASTRUCTURE ONLY. Nothing in the product library links, loads or
// calls this file; only the tests, the smoke check and the benchmark's CPU
// baseline leg may. It shares no code, header, table or helper with the GPU
// path: it is written directly from the classical rules the paper restates
// and its index conventions, with a sort-based edge map instead of any of
// the GPU path's data structures.
//
// Sources (AlSub, Mlakar et al., ACM TOG; section / equation names):
//   Catmull-Clark rules ............ Sec. 3.1, face-point, edge-point and
//                                    vertex-update equations (eq:pos_update),
//                                    boundary rule (eq::CC_boundary)
//   vertex order of the refined mesh Sec. 3.2 "Topology refinement":
//                                    face point of face r is |v|+r, edge
//                                    point of edge e is |v|+|f|+e
//   edge ids ....................... Sec. 3.2: enumeration of the non-zeros
//                                    of the upper triangle of E (read here
//                                    as ascending (hi, lo), i.e. CSC order)
//   valence ........................ eq:vo (incident faces)
//   creases ........................ Sec. 3.3: crease valency eq:CC_crease_valency,
//                                    vertex sharpness eq:CC_crease_vsharpness,
//                                    Chaikin-type inheritance (two sigma
//                                    equations), crease vertices overwrite
//   sqrt(3) ........................ App. A, equ:sqrt2 and equ:alpha, child
//                                    triangles and index |v|+i of face points
//   Loop ........................... App. B, eq:loop_smooth and beta, the
//                                    1-to-4 split
//   single-SpMV matrix R_k ......... Sec. 3.6 (P_{i+1} = R_i P_i)
//   sqrt(3) boundary ............... App. A leaves the boundary to Kobbelt's
//                                    sqrt(3) paper: a two-step cycle whose
//                                    second step trisects the boundary
//                                    (scheme code 3 below, the "trisection
//                                    step"; the first step of the cycle is
//                                    the sqrt(3) step with fixed boundary)
//
// Readings where the paper is silent (each listed in the design notes):
//   * 0-based ids; -1 = "no face".
//   * Loop edge point = 3/8 (edge ends) + 1/8 (opposite vertices) (the
//     weights live only in a figure of the paper); boundary edge = midpoint,
//     boundary vertex = 3/4 p + 1/8 (two boundary neighbours).
//   * sqrt(3): boundary half-edges are not flipped and emit (v_j, v_j+1, f_r);
//     boundary vertices stay fixed.
//   * Loop/sqrt(3) valence n = number of distinct neighbours.
//   * Creases (Catmull-Clark and Loop; the paper gives them for
//     Catmull-Clark, and Loop takes the same rules on its own smooth
//     points, with Loop's edge point as the "smooth" edge value; sqrt(3)
//     rejects them): k = incident edges with sigma > 0,
//     s = mean of their sigma. Edge: sigma >= 1 -> midpoint, else blend
//     (1-sigma) smooth + sigma midpoint. Vertex: k <= 1 smooth, k == 2 crease
//     rule 3/4 p + 1/8 (a + b), k >= 3 corner p; s >= 1 -> sharp rule, else
//     (1-s) smooth + s sharp. Boundary rules win over creases.
//   * Chaikin neighbour: at an end point with exactly two creases the other
//     crease's sigma, otherwise the crease's own sigma. Sharpness is carried
//     in FP64 with the fixed order 0.25*(si + 3.0*sj) - 1.0 (no contraction,
//     this file is compiled with -ffp-contract=off); a child is kept iff > 0.
//   * Invalid inputs are rejected (status codes below) instead of refined.
//   * sqrt(3) trisection step (the second step of Kobbelt's boundary cycle;
//     the paper defers the boundary rule to that work, so every detail here
//     is a reading): every face has at most one boundary edge (true after a
//     first step, whose boundary faces are (v_j, v_j+1, face point)). A
//     boundary face r with boundary edge j = (u, w) gets no face point;
//     instead its edge is trisected by p (near u, index |v| + r) and q (near
//     w, index |v| + |f| + rank of r among the boundary faces). Its children
//     are 3r+j = (p, q, v_j+2), 3r+j+1 = (v_j+1, X, q), 3r+j+2 = (v_j+2, X, p);
//     p and q stand in for the missing face point wherever a neighbour's
//     flipped edge would reach it (q across edge j+1, p across edge j+2).
//     Boundary points follow the ternary subdivision of a uniform cubic
//     B-spline curve (mask [1 4 10 16 19 16 10 4 1] / 27): p = (u- + 16 u +
//     10 w) / 27, q = (10 u + 16 w + w+) / 27, old boundary vertex
//     (4 a + 19 v + 4 b) / 27 over its boundary neighbours; interior
//     vertices and face points as in the sqrt(3) step.
#include <algorithm>
#include <cmath>
#include <cstdint>
#include <cstring>
#include <utility>
#include <vector>

namespace {

enum Scheme { CATMULL_CLARK = 0, LOOP = 1, SQRT3 = 2, SQRT3_TRISECT = 3 };

// Fault flags; the reported status is the first set flag in this order.
enum Fault {
  F_INVALID_ARG = 1,
  F_SCHEME_MESH = 2,
  F_DEGENERATE = 4,
  F_NONMANIFOLD = 8,
  F_BAD_CREASE = 16,
};

int status_of(unsigned flags) {
  if (flags & F_INVALID_ARG) return -1;
  if (flags & F_SCHEME_MESH) return -2;
  if (flags & F_DEGENERATE) return -4;
  if (flags & F_NONMANIFOLD) return -3;
  if (flags & F_BAD_CREASE) return -5;
  return 0;
}

// ---------------------------------------------------------------- values
// A refined vertex value is either a 3-vector of positions or a sparse row
// of weights over the coarse vertices (used to assemble R_k). The rules are
// written once against these two operations.
struct Vec3 {
  double x = 0, y = 0, z = 0;
};
inline void acc(Vec3& d, double w, const Vec3& s) {
  d.x += w * s.x;
  d.y += w * s.y;
  d.z += w * s.z;
}

struct Row {
  std::vector<std::pair<int, double>> e;  // (coarse vertex, weight)
};
inline void acc(Row& d, double w, const Row& s) {
  for (const auto& p : s.e) d.e.emplace_back(p.first, w * p.second);
}
inline void compact(Row& r) {
  std::sort(r.e.begin(), r.e.end(),
            [](const std::pair<int, double>& a, const std::pair<int, double>& b) { return a.first < b.first; });
  std::vector<std::pair<int, double>> out;
  for (const auto& p : r.e) {
    if (!out.empty() && out.back().first == p.first)
      out.back().second += p.second;
    else
      out.push_back(p);
  }
  r.e.swap(out);
}

// ---------------------------------------------------------------- topology
struct Level {
  int nv = 0;
  std::vector<int> off;  // F+1 column pointer of the mesh matrix
  std::vector<int> fv;   // H row indices, CCW per face
  int nf() const { return (int)off.size() - 1; }
  int nh() const { return (int)fv.size(); }
};

struct Crease {
  int lo, hi;
  double sigma;
};

struct HalfEdge {
  int hi, lo, face, slot, from;
};

// Per-vertex lists stored flat: items of vertex v are item[ptr[v] .. ptr[v+1]).
struct VertexLists {
  std::vector<int64_t> ptr;
  std::vector<int> item;
  int size(int v) const { return (int)(ptr[v + 1] - ptr[v]); }
  const int* begin(int v) const { return item.data() + ptr[v]; }
  const int* end(int v) const { return item.data() + ptr[v + 1]; }
  int at(int v, int i) const { return item[ptr[v] + i]; }
};

// Build lists from (vertex, item) pairs, keeping the pairs' order per vertex.
VertexLists group_by_vertex(int V, const std::vector<std::pair<int, int>>& pairs) {
  VertexLists L;
  L.ptr.assign((size_t)V + 1, 0);
  for (const auto& p : pairs) L.ptr[p.first + 1]++;
  for (int v = 0; v < V; ++v) L.ptr[v + 1] += L.ptr[v];
  L.item.resize(pairs.size());
  std::vector<int64_t> fill(L.ptr.begin(), L.ptr.end() - 1);
  for (const auto& p : pairs) L.item[fill[p.first]++] = p.second;
  return L;
}

// Adjacency of one level, derived by sorting half-edges.
struct Adjacency {
  unsigned faults = 0;
  int ne = 0;
  std::vector<int> he_face;           // per half-edge: its face
  std::vector<int> he_eid;            // per half-edge: edge id
  std::vector<int> e_lo, e_hi;        // per edge: endpoints (eid order)
  std::vector<int> e_he0, e_he1;      // per edge: its half-edges (he1 = -1: boundary)
  std::vector<int> valence;           // per vertex: incident faces (eq:vo)
  VertexLists nbrs;                   // per vertex: distinct neighbours
  VertexLists bnd;                    // per vertex: other ends of its boundary edges
  VertexLists vfaces;                 // per vertex: incident faces
  VertexLists corners;                // per vertex: its half-edges (corners)
};

int he_next(const Level& L, int f, int h) { return h + 1 == L.off[f + 1] ? L.off[f] : h + 1; }
int he_prev(const Level& L, int f, int h) { return h == L.off[f] ? L.off[f + 1] - 1 : h - 1; }

Adjacency analyse(const Level& L) {
  Adjacency A;
  const int F = L.nf(), H = L.nh(), V = L.nv;
  A.he_face.assign(H, -1);
  A.he_eid.assign(H, -1);
  // faces: order >= 3, indices in range, no repeated vertex
  for (int f = 0; f < F; ++f) {
    const int b = L.off[f], e = L.off[f + 1];
    if (e - b < 3) A.faults |= F_DEGENERATE;
    for (int h = b; h < e; ++h) {
      A.he_face[h] = f;
      if (L.fv[h] < 0 || L.fv[h] >= V) A.faults |= F_INVALID_ARG;
      for (int g = b; g < h; ++g)
        if (L.fv[g] == L.fv[h]) A.faults |= F_DEGENERATE;
    }
  }
  if (A.faults) return A;
  // half-edges keyed by (hi, lo); sort gives the edge enumeration
  std::vector<HalfEdge> hes(H);
  for (int f = 0; f < F; ++f)
    for (int h = L.off[f]; h < L.off[f + 1]; ++h) {
      int a = L.fv[h], b = L.fv[he_next(L, f, h)];
      hes[h] = HalfEdge{std::max(a, b), std::min(a, b), f, h - L.off[f], a};
    }
  std::sort(hes.begin(), hes.end(), [](const HalfEdge& x, const HalfEdge& y) {
    if (x.hi != y.hi) return x.hi < y.hi;
    if (x.lo != y.lo) return x.lo < y.lo;
    if (x.face != y.face) return x.face < y.face;
    return x.slot < y.slot;
  });
  for (int i = 0; i < H;) {
    int j = i;
    while (j < H && hes[j].hi == hes[i].hi && hes[j].lo == hes[i].lo) ++j;
    const int eid = A.ne++;
    A.e_lo.push_back(hes[i].lo);
    A.e_hi.push_back(hes[i].hi);
    const int h0 = L.off[hes[i].face] + hes[i].slot;
    int h1 = -1;
    if (j - i > 2) A.faults |= F_NONMANIFOLD;
    if (j - i == 2) {
      h1 = L.off[hes[i + 1].face] + hes[i + 1].slot;
      if (hes[i].from == hes[i + 1].from) A.faults |= F_NONMANIFOLD;  // same direction twice
    }
    A.e_he0.push_back(h0);
    A.e_he1.push_back(h1);
    for (int k = i; k < j; ++k) A.he_eid[L.off[hes[k].face] + hes[k].slot] = eid;
    i = j;
  }
  // per-vertex data
  A.valence.assign(V, 0);
  std::vector<std::pair<int, int>> nb, bd, vf, co;
  nb.reserve((size_t)2 * A.ne);
  vf.reserve(H);
  co.reserve(H);
  for (int h = 0; h < H; ++h) {
    A.valence[L.fv[h]]++;
    vf.emplace_back(L.fv[h], A.he_face[h]);
    co.emplace_back(L.fv[h], h);
  }
  for (int e = 0; e < A.ne; ++e) {
    nb.emplace_back(A.e_lo[e], A.e_hi[e]);
    nb.emplace_back(A.e_hi[e], A.e_lo[e]);
    if (A.e_he1[e] < 0) {
      bd.emplace_back(A.e_lo[e], A.e_hi[e]);
      bd.emplace_back(A.e_hi[e], A.e_lo[e]);
    }
  }
  A.nbrs = group_by_vertex(V, nb);
  A.bnd = group_by_vertex(V, bd);
  A.vfaces = group_by_vertex(V, vf);
  A.corners = group_by_vertex(V, co);
  for (int v = 0; v < V; ++v)
    if (A.valence[v] == 0) A.faults |= F_DEGENERATE;  // isolated vertex
  // one fan per vertex: the corners around v must be connected through
  // shared edges (catches "bow-tie" and pinched vertices)
  std::vector<int> comp;
  for (int v = 0; v < V; ++v) {
    const int n = A.corners.size(v);
    if (n == 0) continue;
    const int* c = A.corners.begin(v);
    comp.resize(n);
    for (int i = 0; i < n; ++i) comp[i] = i;
    bool changed = true;
    while (changed) {
      changed = false;
      for (int i = 0; i < n; ++i) {
        const int out_i = L.fv[he_next(L, A.he_face[c[i]], c[i])];
        for (int j = 0; j < n; ++j) {
          const int in_j = L.fv[he_prev(L, A.he_face[c[j]], c[j])];
          if (out_i == in_j) {
            const int m = std::min(comp[i], comp[j]);
            if (comp[i] != m || comp[j] != m) {
              comp[i] = comp[j] = m;
              changed = true;
            }
          }
        }
      }
    }
    for (int i = 0; i < n; ++i)
      if (comp[i] != 0) A.faults |= F_NONMANIFOLD;
  }
  return A;
}

// ---------------------------------------------------------------- creases
// Edge-indexed sharpness of the creases of one level; 0 = smooth edge.
unsigned crease_table(const Adjacency& A, const std::vector<Crease>& cr, std::vector<double>& sig) {
  unsigned faults = 0;
  sig.assign(A.ne, 0.0);
  std::vector<char> seen(A.ne, 0);
  for (const Crease& c : cr) {
    if (!(c.sigma >= 0.0) || std::isinf(c.sigma) || c.lo == c.hi) {
      faults |= F_BAD_CREASE;
      continue;
    }
    const int lo = std::min(c.lo, c.hi), hi = std::max(c.lo, c.hi);
    // edges are sorted by (hi, lo): binary search
    int a = 0, b = A.ne;
    while (a < b) {
      const int m = (a + b) / 2;
      if (A.e_hi[m] < hi || (A.e_hi[m] == hi && A.e_lo[m] < lo))
        a = m + 1;
      else
        b = m;
    }
    if (a >= A.ne || A.e_hi[a] != hi || A.e_lo[a] != lo || seen[a]) {
      faults |= F_BAD_CREASE;
      continue;
    }
    seen[a] = 1;
    sig[a] = c.sigma;
  }
  return faults;
}

double chaikin(double si, double sj) {
  const double t = 0.25 * (si + 3.0 * sj) - 1.0;
  return t > 0.0 ? t : 0.0;
}

// ---------------------------------------------------------------- the step
struct Result {
  int status = 0;
  int scheme = 0;
  Level out;
  std::vector<Vec3> P;
  std::vector<Crease> creases;
  // input-level adjacency exported for topology parity
  std::vector<int> e_lo, e_hi;
  int n_boundary = 0;
  // R_k in CSR, if requested
  std::vector<int64_t> r_ptr;
  std::vector<int> r_col;
  std::vector<double> r_val;
};

// Boundary faces of a trisection step: slot of the face's boundary edge (or
// -1) and the face's rank among the boundary faces (face order). Faults when
// a face has more than one boundary edge.
struct BoundaryFaces {
  std::vector<int> slot, rank;
  int count = 0;
  unsigned faults = 0;
};
BoundaryFaces boundary_faces(const Level& L, const Adjacency& A) {
  BoundaryFaces b;
  b.slot.assign(L.nf(), -1);
  b.rank.assign(L.nf(), -1);
  for (int r = 0; r < L.nf(); ++r) {
    int n = 0;
    for (int h = L.off[r]; h < L.off[r + 1]; ++h) {
      const int e = A.he_eid[h];
      if (A.e_he1[e] < 0) {
        b.slot[r] = h - L.off[r];
        ++n;
      }
    }
    if (n > 1) b.faults |= F_INVALID_ARG;
    if (n == 1) b.rank[r] = b.count++;
  }
  return b;
}

// the boundary neighbour of boundary vertex v other than w
int other_boundary_nbr(const Adjacency& A, int v, int w) {
  return A.bnd.at(v, 0) == w ? A.bnd.at(v, 1) : A.bnd.at(v, 0);
}

template <class T>
struct Evaluator {
  // Vertex data of the refined level, from vertex data of this level.
  const Level& L;
  const Adjacency& A;
  const std::vector<double>& sig;  // per edge
  int scheme;

  std::vector<T> face_points(const std::vector<T>& P) const {
    std::vector<T> f(L.nf());
    for (int r = 0; r < L.nf(); ++r) {
      const int c = L.off[r + 1] - L.off[r];
      for (int h = L.off[r]; h < L.off[r + 1]; ++h) acc(f[r], 1.0 / c, P[L.fv[h]]);
    }
    return f;
  }

  // vertex of face(h) opposite to half-edge h (triangles)
  int opposite(int h) const {
    const int f = A.he_face[h];
    return L.fv[he_prev(L, f, h)];
  }

  // Crease vertices overwrite the smooth vertex points out[0..V): crease
  // valency k (eq:CC_crease_valency) and vertex sharpness s, the mean of the
  // incident creases' sigma (eq:CC_crease_vsharpness); k == 2 takes the
  // crease rule 3/4 p + 1/8 (the two crease neighbours), k >= 3 the corner
  // rule p, blended with the smooth point when s < 1. Boundary vertices keep
  // the boundary rule. The same rules serve Catmull-Clark and Loop.
  void crease_vertices(const std::vector<T>& P, std::vector<T>& out) const {
    const int V = L.nv, E = A.ne;
    std::vector<int> k(V, 0);
    std::vector<double> ssum(V, 0.0);
    std::vector<std::vector<int>> cnb(V);
    for (int e = 0; e < E; ++e)
      if (sig[e] > 0.0) {
        for (int end = 0; end < 2; ++end) {
          const int v = end ? A.e_hi[e] : A.e_lo[e];
          const int w = end ? A.e_lo[e] : A.e_hi[e];
          k[v]++;
          ssum[v] += sig[e];
          cnb[v].push_back(w);
        }
      }
    for (int v = 0; v < V; ++v) {
      if (A.bnd.size(v) > 0 || k[v] < 2) continue;
      T sharp;
      if (k[v] == 2) {
        acc(sharp, 0.75, P[v]);
        acc(sharp, 0.125, P[cnb[v][0]]);
        acc(sharp, 0.125, P[cnb[v][1]]);
      } else {
        acc(sharp, 1.0, P[v]);
      }
      const double s = ssum[v] / k[v];
      if (s >= 1.0) {
        out[v] = sharp;
      } else {
        T blend;
        acc(blend, 1.0 - s, out[v]);
        acc(blend, s, sharp);
        out[v] = blend;
      }
    }
  }

  // An interior crease edge's point: sigma >= 1 the midpoint, 0 < sigma < 1
  // (1 - sigma) smooth + sigma midpoint.
  void crease_edge(double s, const T& smooth, const T& pa, const T& pb, T& ep) const {
    if (s >= 1.0) {
      acc(ep, 0.5, pa);
      acc(ep, 0.5, pb);
    } else if (s > 0.0) {
      T mid;
      acc(mid, 0.5, pa);
      acc(mid, 0.5, pb);
      acc(ep, 1.0 - s, smooth);
      acc(ep, s, mid);
    } else {
      ep = smooth;
    }
  }

  std::vector<T> run(const std::vector<T>& P) const {
    const int V = L.nv, F = L.nf(), E = A.ne;
    std::vector<T> out;
    if (scheme == CATMULL_CLARK) {
      const std::vector<T> f = face_points(P);
      out.resize((size_t)V + F + E);
      // vertex points (eq:pos_update split as s1 + s2 + s3)
      for (int v = 0; v < V; ++v) {
        T& S = out[v];
        if (A.bnd.size(v) > 0) {  // eq::CC_boundary
          acc(S, 0.75, P[v]);
          acc(S, 0.125, P[A.bnd.at(v, 0)]);
          acc(S, 0.125, P[A.bnd.at(v, 1)]);
          continue;
        }
        const double n = A.valence[v];
        acc(S, 1.0 - 2.0 / n, P[v]);                              // s1
        for (const int* w = A.nbrs.begin(v); w != A.nbrs.end(v); ++w) acc(S, 1.0 / (n * n), P[*w]);  // s2
        for (const int* r = A.vfaces.begin(v); r != A.vfaces.end(v); ++r) acc(S, 1.0 / (n * n), f[*r]);  // s3
      }
      crease_vertices(P, out);
      for (int r = 0; r < F; ++r) out[(size_t)V + r] = f[r];
      // edge points
      for (int e = 0; e < E; ++e) {
        T& ep = out[(size_t)V + F + e];
        const int a = A.e_lo[e], b = A.e_hi[e];
        if (A.e_he1[e] < 0) {
          acc(ep, 0.5, P[a]);
          acc(ep, 0.5, P[b]);
          continue;
        }
        T smooth;
        acc(smooth, 0.25, P[a]);
        acc(smooth, 0.25, P[b]);
        acc(smooth, 0.25, f[A.he_face[A.e_he0[e]]]);
        acc(smooth, 0.25, f[A.he_face[A.e_he1[e]]]);
        crease_edge(sig[e], smooth, P[a], P[b], ep);
      }
    } else if (scheme == LOOP) {
      out.resize((size_t)V + E);
      for (int v = 0; v < V; ++v) {
        T& S = out[v];
        if (A.bnd.size(v) > 0) {
          acc(S, 0.75, P[v]);
          acc(S, 0.125, P[A.bnd.at(v, 0)]);
          acc(S, 0.125, P[A.bnd.at(v, 1)]);
          continue;
        }
        const double n = (double)A.nbrs.size(v);
        const double c = 3.0 / 8.0 + 0.25 * std::cos(2.0 * M_PI / n);
        const double beta = (5.0 / 8.0 - c * c) / n;
        acc(S, 1.0 - n * beta, P[v]);
        for (const int* w = A.nbrs.begin(v); w != A.nbrs.end(v); ++w) acc(S, beta, P[*w]);
      }
      crease_vertices(P, out);  // the crease rules of Catmull-Clark, applied to Loop's points
      for (int e = 0; e < E; ++e) {
        T& ep = out[(size_t)V + e];
        const int a = A.e_lo[e], b = A.e_hi[e];
        if (A.e_he1[e] < 0) {
          acc(ep, 0.5, P[a]);
          acc(ep, 0.5, P[b]);
          continue;
        }
        T smooth;
        acc(smooth, 0.375, P[a]);
        acc(smooth, 0.375, P[b]);
        acc(smooth, 0.125, P[opposite(A.e_he0[e])]);
        acc(smooth, 0.125, P[opposite(A.e_he1[e])]);
        crease_edge(sig[e], smooth, P[a], P[b], ep);
      }
    } else if (scheme == SQRT3_TRISECT) {
      const BoundaryFaces bf = boundary_faces(L, A);
      const std::vector<T> f = face_points(P);
      out.resize((size_t)V + F + bf.count);
      for (int v = 0; v < V; ++v) {
        T& S = out[v];
        if (A.bnd.size(v) > 0) {  // ternary cubic B-spline rule on the boundary polygon
          acc(S, 4.0 / 27.0, P[A.bnd.at(v, 0)]);
          acc(S, 19.0 / 27.0, P[v]);
          acc(S, 4.0 / 27.0, P[A.bnd.at(v, 1)]);
          continue;
        }
        const double n = (double)A.nbrs.size(v);
        const double alpha = (4.0 - 2.0 * std::cos(2.0 * M_PI / n)) / 9.0;
        acc(S, 1.0 - alpha, P[v]);
        for (const int* w = A.nbrs.begin(v); w != A.nbrs.end(v); ++w) acc(S, alpha / n, P[*w]);
      }
      for (int r = 0; r < F; ++r) {
        if (bf.slot[r] < 0) {
          out[(size_t)V + r] = f[r];
          continue;
        }
        const int j = bf.slot[r];
        const int u = L.fv[L.off[r] + j], w = L.fv[L.off[r] + (j + 1) % 3];
        const int um = other_boundary_nbr(A, u, w), wp = other_boundary_nbr(A, w, u);
        T& p = out[(size_t)V + r];
        acc(p, 1.0 / 27.0, P[um]);
        acc(p, 16.0 / 27.0, P[u]);
        acc(p, 10.0 / 27.0, P[w]);
        T& q = out[(size_t)V + F + bf.rank[r]];
        acc(q, 10.0 / 27.0, P[u]);
        acc(q, 16.0 / 27.0, P[w]);
        acc(q, 1.0 / 27.0, P[wp]);
      }
    } else {  // SQRT3
      const std::vector<T> f = face_points(P);
      out.resize((size_t)V + F);
      for (int v = 0; v < V; ++v) {
        T& S = out[v];
        if (A.bnd.size(v) > 0) {
          acc(S, 1.0, P[v]);
          continue;
        }
        const double n = (double)A.nbrs.size(v);
        const double alpha = (4.0 - 2.0 * std::cos(2.0 * M_PI / n)) / 9.0;
        acc(S, 1.0 - alpha, P[v]);
        for (const int* w = A.nbrs.begin(v); w != A.nbrs.end(v); ++w) acc(S, alpha / n, P[*w]);
      }
      for (int r = 0; r < F; ++r) out[(size_t)V + r] = f[r];
    }
    return out;
  }
};

// Crease inheritance (Chaikin variant): crease edge e = (lo, hi) has the
// children (lo, m) and (hi, m), m = first_ep + e its edge point, with the
// sharpness of the rule at each end; children of sharpness 0 are dropped.
// Sorted by (hi, lo) like the edge ids.
void inherit_creases(int V, int first_ep, const Adjacency& A, const std::vector<double>& sig, Result& R) {
  const int E = A.ne;
  std::vector<int> k(V, 0);
  std::vector<std::vector<int>> ce(V);
  for (int e = 0; e < E; ++e)
    if (sig[e] > 0.0) {
      k[A.e_lo[e]]++;
      k[A.e_hi[e]]++;
      ce[A.e_lo[e]].push_back(e);
      ce[A.e_hi[e]].push_back(e);
    }
  for (int e = 0; e < E; ++e) {
    if (!(sig[e] > 0.0)) continue;
    const int m = first_ep + e;
    for (int end = 0; end < 2; ++end) {
      const int v = end ? A.e_hi[e] : A.e_lo[e];
      double si = sig[e];
      if (k[v] == 2) si = sig[ce[v][0] == e ? ce[v][1] : ce[v][0]];
      const double sc = chaikin(si, sig[e]);
      if (sc > 0.0) R.creases.push_back(Crease{v, m, sc});  // lo = v < hi = m
    }
  }
  std::sort(R.creases.begin(), R.creases.end(), [](const Crease& x, const Crease& y) {
    return x.hi != y.hi ? x.hi < y.hi : x.lo < y.lo;
  });
}

// Topology of the refined mesh and inherited creases.
void refine_topology(int scheme, const Level& L, const Adjacency& A, const std::vector<double>& sig, Result& R) {
  const int V = L.nv, F = L.nf(), H = L.nh(), E = A.ne;
  Level& O = R.out;
  if (scheme == CATMULL_CLARK) {
    // column r of M becomes c_r quads; child (r, j) sits at off_r + j
    O.nv = V + F + E;
    O.off.resize((size_t)H + 1);
    O.fv.resize((size_t)4 * H);
    for (int i = 0; i <= H; ++i) O.off[i] = 4 * i;
    for (int r = 0; r < F; ++r)
      for (int h = L.off[r]; h < L.off[r + 1]; ++h) {
        const int hp = he_prev(L, r, h);
        int* q = &O.fv[(size_t)4 * h];
        q[0] = L.fv[h];
        q[1] = V + F + A.he_eid[h];
        q[2] = V + r;
        q[3] = V + F + A.he_eid[hp];
      }
    inherit_creases(V, V + F, A, sig, R);
  } else if (scheme == LOOP) {
    O.nv = V + E;
    O.off.resize((size_t)4 * F + 1);
    O.fv.resize((size_t)12 * F);
    for (int i = 0; i <= 4 * F; ++i) O.off[i] = 3 * i;
    for (int r = 0; r < F; ++r) {
      const int b = L.off[r];
      int e[3];
      for (int j = 0; j < 3; ++j) e[j] = V + A.he_eid[b + j];
      for (int j = 0; j < 3; ++j) {
        int* t = &O.fv[(size_t)3 * (4 * r + j)];
        t[0] = L.fv[b + j];
        t[1] = e[j];
        t[2] = e[(j + 2) % 3];
      }
      int* t = &O.fv[(size_t)3 * (4 * r + 3)];
      t[0] = e[0];
      t[1] = e[1];
      t[2] = e[2];
    }
    inherit_creases(V, V, A, sig, R);
  } else if (scheme == SQRT3_TRISECT) {
    const BoundaryFaces bf = boundary_faces(L, A);
    O.nv = V + F + bf.count;
    O.off.resize((size_t)3 * F + 1);
    O.fv.resize((size_t)9 * F);
    for (int i = 0; i <= 3 * F; ++i) O.off[i] = 3 * i;
    // the point of face s that its neighbour across s's edge i links to: the
    // face point, or on a boundary face q (edge j+1) or p (edge j+2)
    auto link = [&](int s, int i) {
      const int js = bf.slot[s];
      if (js < 0) return V + s;
      return i == (js + 1) % 3 ? V + F + bf.rank[s] : V + s;
    };
    for (int r = 0; r < F; ++r) {
      const int b = L.off[r];
      int X[3];  // across edge i: the neighbour's linked point (boundary edge: unused)
      for (int i = 0; i < 3; ++i) {
        const int e = A.he_eid[b + i];
        const int other = A.e_he0[e] == b + i ? A.e_he1[e] : A.e_he0[e];
        X[i] = other >= 0 ? link(A.he_face[other], other - L.off[A.he_face[other]]) : -1;
      }
      const int j = bf.slot[r];
      for (int i = 0; i < 3; ++i) {
        int* t = &O.fv[(size_t)3 * (b + i)];
        if (j < 0) {
          t[0] = L.fv[b + i];
          t[1] = X[i];
          t[2] = V + r;
        } else if (i == j) {  // (p, q, v_j+2)
          t[0] = V + r;
          t[1] = V + F + bf.rank[r];
          t[2] = L.fv[b + (j + 2) % 3];
        } else if (i == (j + 1) % 3) {  // (v_j+1, X, q)
          t[0] = L.fv[b + i];
          t[1] = X[i];
          t[2] = V + F + bf.rank[r];
        } else {  // (v_j+2, X, p)
          t[0] = L.fv[b + i];
          t[1] = X[i];
          t[2] = V + r;
        }
      }
    }
  } else {
    O.nv = V + F;
    O.off.resize((size_t)3 * F + 1);
    O.fv.resize((size_t)9 * F);
    for (int i = 0; i <= 3 * F; ++i) O.off[i] = 3 * i;
    for (int r = 0; r < F; ++r)
      for (int j = 0; j < 3; ++j) {
        const int h = L.off[r] + j;
        const int e = A.he_eid[h];
        const int other = A.e_he0[e] == h ? A.e_he1[e] : A.e_he0[e];
        int* t = &O.fv[(size_t)3 * h];
        t[0] = L.fv[h];
        t[1] = other >= 0 ? V + A.he_face[other] : L.fv[he_next(L, r, h)];
        t[2] = V + r;
      }
  }
}

}  // namespace

extern "C" {

// One refinement step of the mesh (nv vertices; nf faces with column pointer
// `off` [nf+1] and row indices `fv` [off[nf]]; positions P [nv*3]; nc creases
// with end points cv [2*nc] and sharpness cs [nc]). If want_R != 0 the
// refinement matrix R_k is assembled as well. Returns an owned handle (free
// with oracle_free) and the status in *status (0 ok, <0 as in the design notes).
void* oracle_step(int scheme, int nv, int nf, const int* off, const int* fv, const double* P, int nc,
                  const int* cv, const double* cs, int want_R, int* status) {
  Result* R = new Result();
  R->scheme = scheme;
  unsigned faults = 0;
  if (scheme < 0 || scheme > 3 || nv < 0 || nf < 0 || nc < 0) faults |= F_INVALID_ARG;
  Level L;
  L.nv = nv;
  if (!faults) {
    L.off.assign(off, off + nf + 1);
    if (L.off[0] != 0) faults |= F_INVALID_ARG;
    for (int f = 0; f < nf; ++f)
      if (L.off[f + 1] < L.off[f]) faults |= F_INVALID_ARG;
  }
  if (!faults) {
    L.fv.assign(fv, fv + L.off[nf]);
    if (scheme != CATMULL_CLARK) {
      for (int f = 0; f < nf; ++f)
        if (L.off[f + 1] - L.off[f] != 3) faults |= F_SCHEME_MESH;
      if (nc > 0 && (scheme == SQRT3 || scheme == SQRT3_TRISECT))
        faults |= F_INVALID_ARG;  // creases: Catmull-Clark and Loop
    }
  }
  Adjacency A;
  std::vector<double> sig;
  if (!faults) {
    A = analyse(L);
    faults |= A.faults;
  }
  if (!faults && scheme == SQRT3_TRISECT) faults |= boundary_faces(L, A).faults;
  if (!faults) {
    std::vector<Crease> cr;
    for (int i = 0; i < nc; ++i) {
      if (cv[2 * i] < 0 || cv[2 * i] >= nv || cv[2 * i + 1] < 0 || cv[2 * i + 1] >= nv) {
        faults |= F_BAD_CREASE;
        continue;
      }
      if (cs[i] == 0.0) continue;  // sharpness 0: a smooth edge
      cr.push_back(Crease{cv[2 * i], cv[2 * i + 1], cs[i]});
    }
    faults |= crease_table(A, cr, sig);
    if (cr.empty()) sig.assign(A.ne, 0.0);
  }
  R->status = status_of(faults);
  *status = R->status;
  if (R->status != 0) return R;

  R->e_lo = A.e_lo;
  R->e_hi = A.e_hi;
  for (int e = 0; e < A.ne; ++e) R->n_boundary += A.e_he1[e] < 0;
  refine_topology(scheme, L, A, sig, *R);

  std::vector<Vec3> Pin(nv);
  for (int v = 0; v < nv; ++v) Pin[v] = Vec3{P[3 * v], P[3 * v + 1], P[3 * v + 2]};
  Evaluator<Vec3> ev3{L, A, sig, scheme};
  R->P = ev3.run(Pin);

  if (want_R) {
    std::vector<Row> I(nv);
    for (int v = 0; v < nv; ++v) I[v].e.emplace_back(v, 1.0);
    Evaluator<Row> evr{L, A, sig, scheme};
    std::vector<Row> rows = evr.run(I);
    R->r_ptr.assign(rows.size() + 1, 0);
    for (size_t i = 0; i < rows.size(); ++i) {
      compact(rows[i]);
      R->r_ptr[i + 1] = R->r_ptr[i] + (int64_t)rows[i].e.size();
    }
    R->r_col.reserve(R->r_ptr.back());
    R->r_val.reserve(R->r_ptr.back());
    for (auto& r : rows)
      for (auto& p : r.e) {
        R->r_col.push_back(p.first);
        R->r_val.push_back(p.second);
      }
  }
  return R;
}

// counts: [0] V' [1] F' [2] H' [3] creases' [4] E (input level) [5] boundary
// edges (input level) [6] nnz(R_k) (0 if not assembled)
void oracle_counts(void* h, int64_t* c) {
  const Result* R = (const Result*)h;
  c[0] = R->out.nv;
  c[1] = R->out.nf();
  c[2] = R->out.nh();
  c[3] = (int64_t)R->creases.size();
  c[4] = (int64_t)R->e_lo.size();
  c[5] = R->n_boundary;
  c[6] = R->r_ptr.empty() ? 0 : R->r_ptr.back();
}

void oracle_mesh(void* h, int* off, int* fv, double* P) {
  const Result* R = (const Result*)h;
  std::memcpy(off, R->out.off.data(), R->out.off.size() * sizeof(int));
  std::memcpy(fv, R->out.fv.data(), R->out.fv.size() * sizeof(int));
  for (size_t v = 0; v < R->P.size(); ++v) {
    P[3 * v] = R->P[v].x;
    P[3 * v + 1] = R->P[v].y;
    P[3 * v + 2] = R->P[v].z;
  }
}

void oracle_edges(void* h, int* lohi) {
  const Result* R = (const Result*)h;
  for (size_t e = 0; e < R->e_lo.size(); ++e) {
    lohi[2 * e] = R->e_lo[e];
    lohi[2 * e + 1] = R->e_hi[e];
  }
}

void oracle_creases(void* h, int* cv, double* cs) {
  const Result* R = (const Result*)h;
  for (size_t i = 0; i < R->creases.size(); ++i) {
    cv[2 * i] = R->creases[i].lo;
    cv[2 * i + 1] = R->creases[i].hi;
    cs[i] = R->creases[i].sigma;
  }
}

void oracle_R(void* h, int64_t* ptr, int* col, double* val) {
  const Result* R = (const Result*)h;
  std::memcpy(ptr, R->r_ptr.data(), R->r_ptr.size() * sizeof(int64_t));
  std::memcpy(col, R->r_col.data(), R->r_col.size() * sizeof(int));
  std::memcpy(val, R->r_val.data(), R->r_val.size() * sizeof(double));
}

void oracle_free(void* h) { delete (Result*)h; }

}  // extern "C"
