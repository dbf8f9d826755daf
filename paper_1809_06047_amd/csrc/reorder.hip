// Mesh reordering (Sec. 4.5): reverse Cuthill-McKee on the vertex graph of a
// cage, rows of M permuted by it, faces sorted by their first non-zero (the
// smallest new id among their corners). A build-step preprocessing of the
// input on the host: the breadth-first order is sequential by definition,
// and the result only changes where the cage's rows and columns sit in HBM.
//
// Fixed here (the paper leaves them open): each connected component starts
// at its unvisited vertex of smallest degree (smaller id first); a dequeued
// vertex appends its unvisited neighbours by increasing (degree, id); the
// whole sequence is reversed; faces are ordered by (first non-zero, old id)
// and keep their corners in cyclic order. Degree = distinct neighbours.
#include <algorithm>
#include <cstdint>
#include <vector>

#include "subdiv_internal.h"

extern "C" int subdiv_rcm_order(int32_t num_vertices, int32_t num_faces, const int32_t *face_offsets,
                                int32_t face_order, const int32_t *face_verts, int32_t *vertex_perm,
                                int32_t *face_perm) {
  const int V = num_vertices, F = num_faces;
  if (V < 1 || F < 1 || !face_verts || !vertex_perm || !face_perm) return SUBDIV_INVALID_ARG;
  if (!face_offsets && face_order < 3) return SUBDIV_INVALID_ARG;
  auto fb = [&](int f) { return face_offsets ? face_offsets[f] : f * face_order; };
  auto fe = [&](int f) { return face_offsets ? face_offsets[f + 1] : (f + 1) * face_order; };
  if (face_offsets) {
    if (face_offsets[0] != 0) return SUBDIV_INVALID_ARG;
    for (int f = 0; f < F; ++f)
      if (face_offsets[f + 1] - face_offsets[f] < 3) return SUBDIV_INVALID_ARG;
  }
  // vertex graph as sorted, distinct adjacency lists (CSR)
  std::vector<int64_t> cnt(V + 1, 0);
  for (int f = 0; f < F; ++f) {
    const int b = fb(f), e = fe(f);
    for (int h = b; h < e; ++h) {
      const int a = face_verts[h], c = face_verts[h + 1 == e ? b : h + 1];
      if (a < 0 || a >= V || c < 0 || c >= V) return SUBDIV_INVALID_ARG;
      ++cnt[a + 1];
      ++cnt[c + 1];
    }
  }
  for (int v = 0; v < V; ++v) cnt[v + 1] += cnt[v];
  std::vector<int32_t> adj(cnt[V]);
  std::vector<int64_t> fill(cnt.begin(), cnt.end() - 1);
  for (int f = 0; f < F; ++f) {
    const int b = fb(f), e = fe(f);
    for (int h = b; h < e; ++h) {
      const int a = face_verts[h], c = face_verts[h + 1 == e ? b : h + 1];
      adj[fill[a]++] = c;
      adj[fill[c]++] = a;
    }
  }
  std::vector<int64_t> start(V + 1, 0);
  std::vector<int32_t> deg(V);
  {
    int64_t out = 0;
    for (int v = 0; v < V; ++v) {
      auto first = adj.begin() + cnt[v], last = adj.begin() + cnt[v + 1];
      std::sort(first, last);
      const auto end = std::unique(first, last);
      start[v] = out;
      for (auto it = first; it != end; ++it) adj[out++] = *it;  // compacts in place (out <= cnt[v])
      deg[v] = (int32_t)(out - start[v]);
    }
    start[V] = out;
  }
  auto before = [&](int a, int b) { return deg[a] != deg[b] ? deg[a] < deg[b] : a < b; };
  // Cuthill-McKee sequence, component by component
  std::vector<int32_t> by_degree(V);
  for (int v = 0; v < V; ++v) by_degree[v] = v;
  std::sort(by_degree.begin(), by_degree.end(), before);
  std::vector<uint8_t> seen(V, 0);
  std::vector<int32_t> seq;
  seq.reserve(V);
  std::vector<int32_t> next;
  for (int s : by_degree) {
    if (seen[s]) continue;
    seen[s] = 1;
    size_t head = seq.size();
    seq.push_back(s);
    while (head < seq.size()) {
      const int v = seq[head++];
      next.clear();
      for (int64_t i = start[v]; i < start[v + 1]; ++i)
        if (!seen[adj[i]]) next.push_back(adj[i]);
      std::sort(next.begin(), next.end(), before);
      for (int w : next) {
        seen[w] = 1;
        seq.push_back(w);
      }
    }
  }
  // reversed: new id V-1-i for the vertex at position i
  std::vector<int32_t> newid(V);
  for (int i = 0; i < V; ++i) {
    vertex_perm[V - 1 - i] = seq[i];
    newid[seq[i]] = V - 1 - i;
  }
  // faces by (smallest new corner, old id)
  std::vector<int32_t> key(F);
  for (int f = 0; f < F; ++f) {
    int k = V;
    for (int h = fb(f); h < fe(f); ++h) k = std::min(k, newid[face_verts[h]]);
    key[f] = k;
  }
  for (int f = 0; f < F; ++f) face_perm[f] = f;
  std::stable_sort(face_perm, face_perm + F, [&](int a, int b) { return key[a] < key[b]; });
  return SUBDIV_OK;
}
