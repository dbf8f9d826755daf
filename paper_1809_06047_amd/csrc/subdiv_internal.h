// Internal declarations shared by the HIP kernels and the host runtime of
// libsubdiv (gfx950). Not part of the public C ABI (include/subdiv.h).
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

#include "../../include/subdiv.h"

namespace subdiv {

// ---- fault flags written by the device validators (atomicOr) -------------
enum : uint32_t {
  FAULT_INVALID_ARG = 1u,
  FAULT_SCHEME_MESH = 2u,
  FAULT_DEGENERATE = 4u,
  FAULT_NONMANIFOLD = 8u,
  FAULT_BAD_CREASE = 16u,
};

// Small block of device-side results the plan reads back.
struct DeviceInfo {
  uint32_t faults;
  int32_t num_edges;          // E of the analysed level (scan total)
  int32_t num_boundary;       // boundary edges
  uint32_t max_sharp_bits;    // float bits of the largest crease sharpness (>= 0 so ordered as uint)
  int32_t max_valence;
  int32_t num_pillows;        // triangles whose three twins lie in one face (two-face components)
  int32_t pad[10];
};

// ---- one level's mesh matrix -------------------------------------------
// Half-edge h is the h-th non-zero of M in CSC order: face f = column, slot j
// = cyclic position, the half-edge runs from fv[h] to fv[next(h)].
struct Topo {
  int32_t V;
  int32_t F;
  int32_t H;
  int32_t order;             // 3 or 4 uniform, 0 = general (off/hface used)
  const int32_t *off;        // [F+1] column pointer (general only)
  const int32_t *hface;      // [H] column of each non-zero (general only)
  const int32_t *fv;         // [H] row indices
};

template <int ORDER>
__device__ __forceinline__ int he_face(const Topo &t, int h) {
  if constexpr (ORDER > 0) return h / ORDER;
  else return t.hface[h];
}
template <int ORDER>
__device__ __forceinline__ int he_next(const Topo &t, int h) {
  if constexpr (ORDER > 0) return (h % ORDER == ORDER - 1) ? h - (ORDER - 1) : h + 1;
  else {
    const int f = t.hface[h];
    return h + 1 == t.off[f + 1] ? t.off[f] : h + 1;
  }
}
template <int ORDER>
__device__ __forceinline__ int he_prev(const Topo &t, int h) {
  if constexpr (ORDER > 0) return (h % ORDER == 0) ? h + (ORDER - 1) : h - 1;
  else {
    const int f = t.hface[h];
    return h == t.off[f] ? t.off[f + 1] - 1 : h - 1;
  }
}
template <int ORDER>
__device__ __forceinline__ int face_begin(const Topo &t, int f) {
  if constexpr (ORDER > 0) return f * ORDER;
  else return t.off[f];
}
template <int ORDER>
__device__ __forceinline__ int face_end(const Topo &t, int f) {
  if constexpr (ORDER > 0) return (f + 1) * ORDER;
  else return t.off[f + 1];
}

// ---- adjacency of one level (the build step's products) ---------------
//   twin[h]  : half-edge opposite to h (F(j,i) of eq:F as a half-edge), -1 on the boundary
//   eid[h]   : id of h's edge (upper triangle of E, ascending (hi, lo))
//   vhe[v]   : one half-edge leaving v; the boundary one if v is on the boundary
//   e2h[e]   : one half-edge of edge e (the lower index of its two)
//   bscan[e] : boundary edges with id < e (only when the level has a boundary)
//   sig[e]   : crease sharpness of edge e (only on levels that may have creases)
//   vcr[v]   : crease valency k and the ids of the first two incident creases
struct Adj {
  int32_t *fv;      // mesh matrix of the level (levels >= 1 only; the cage's is the caller's)
  int32_t *twin;
  int32_t *eid;
  int32_t *vhe;
  int32_t *e2h;
  int32_t *bscan;
  double *sig;
  int4 *vcr;
  int32_t E;
};

// ---- small vector helpers ---------------------------------------------
struct f3 {
  float x, y, z;
};
__device__ __forceinline__ f3 ld3(const float *P, int i) { return *reinterpret_cast<const f3 *>(P + 3ll * i); }
__device__ __forceinline__ void st3(float *P, int i, f3 v) { *reinterpret_cast<f3 *>(P + 3ll * i) = v; }
__device__ __forceinline__ f3 add3(f3 a, f3 b) { return f3{a.x + b.x, a.y + b.y, a.z + b.z}; }
__device__ __forceinline__ f3 mul3(float s, f3 a) { return f3{s * a.x, s * a.y, s * a.z}; }
__device__ __forceinline__ f3 fma3(float s, f3 a, f3 b) { return f3{s * a.x + b.x, s * a.y + b.y, s * a.z + b.z}; }

constexpr int kBlock = 256;

// Stores of the large output streams (face tables, staged point rows) are
// non-temporal: each line is written once and is not read again by the
// kernel that writes it, so it should not displace the rows the kernel
// gathers from L2.
__device__ __forceinline__ void stream_store(uint32_t *p, uint32_t v) { __builtin_nontemporal_store(v, p); }
typedef int v4i32 __attribute__((ext_vector_type(4)));
__device__ __forceinline__ void stream_store4(int4 *p, int4 v) {
  const v4i32 x = {v.x, v.y, v.z, v.w};
  __builtin_nontemporal_store(x, reinterpret_cast<v4i32 *>(p));
}

// A wave's run of dwords lds[0 .. count) to dst[0 .. count), non-temporal:
// 16-byte stores (1 KB per instruction) from the first 16-byte aligned dword
// of dst on, the head before it and the tail after the last whole int4 one
// dword per lane. Against one dword per lane and instruction, this took the
// edge-point runs of cc_edge_group and the last Loop step 5-8% faster.
__device__ __forceinline__ void run_store(const uint32_t *lds, uint32_t *dst, int count, int lane) {
  const int head = min(count, (int)(((16 - (reinterpret_cast<uintptr_t>(dst) & 15)) & 15) >> 2));
  if (lane < head) stream_store(dst + lane, lds[lane]);
  const int body = (count - head) >> 2;
  for (int g = lane; g < body; g += 64) {
    const int d = head + 4 * g;
    stream_store4(reinterpret_cast<int4 *>(dst + d), make_int4(lds[d], lds[d + 1], lds[d + 2], lds[d + 3]));
  }
  const int tail = head + 4 * body;
  if (tail + lane < count) stream_store(dst + tail + lane, lds[tail + lane]);
}

// Coalesced wave stores. A wave whose lane l owns the N dwords
// dst[l*N .. l*N+N) of one contiguous run dst[0 .. 64 N) would store them as
// N per-lane pieces spread over the whole run (one small request per lane
// per instruction). They go through the wave's LDS slice `lds` (64 * (N|1)
// dwords; the odd stride keeps the lane-wise writes conflict-free) and leave
// as N instructions that each write 64 consecutive dwords. `count` = dwords
// of the run that exist (a partial last wave). The stores are non-temporal.
template <int N>
__device__ __forceinline__ void wave_store(uint32_t *lds, const uint32_t (&v)[N], uint32_t *dst, int lane, int count) {
  constexpr int S = N | 1;
#pragma unroll
  for (int k = 0; k < N; ++k) lds[lane * S + k] = v[k];
  __builtin_amdgcn_wave_barrier();
  if constexpr (S == N) {  // odd N: the run is contiguous in LDS too
    run_store(lds, dst, count, lane);
  } else {
#pragma unroll
    for (int t = 0; t < N; ++t) {
      const int g = 64 * t + lane, src = g / N;
      const uint32_t x = lds[src * S + (g - src * N)];
      if (g < count) stream_store(dst + g, x);
    }
  }
  __builtin_amdgcn_wave_barrier();
}

inline unsigned grid_for(long long n, int block = kBlock) {
  long long g = (n + block - 1) / block;
  return (unsigned)(g < 1 ? 1 : g);
}

// ---- launch shapes from the tuning table ------------------------------
// The per-element kernels of the refinement steps are instantiated for
// several workgroup sizes; the tuning table (written by the tuner, loaded by
// the library at its first launch) picks one per kernel and size bucket.
// Every kernel's results are independent of the workgroup size: each lane
// owns its element, and the only cooperation is within a wave (LDS staging of
// stores, shuffles), never across the workgroup.
enum TuneKey {
  TK_LAG_GROUP, TK_LAG_VERTEX, TK_LAG_EDGE, TK_LAG2_GROUP, TK_LAG2_COMBINE, TK_LAG2_OLDER,
  TK_LOOP_EDGE, TK_LOOP_VERTEX, TK_LOOP_FACE, TK_SQRT3_COUNT, TK_SQRT3_FACE, TK_SQRT3_VERTEX,
  TK_LOOPL_FACE, TK_LOOPL_EDGE, TK_SQRT3L_FACE, TK_BW_COEF, TK_BW_FACE, TK_BW_VERTEX,
  TK_COUNT
};
const char *tune_key_name(int key);
// workgroup size for `items` elements of kernel `key` (64, 128, 256 or 512);
// with timing on, the launch is noted for the stage record
int tuned_block(int key, long long items);
// the last tuned launch of this thread since the reset (for the stage timing)
void tune_note_reset();
bool tune_note_take(int *key, long long *items, int *block);
// text for subdiv_last_error() of this thread
void subdiv_set_error(const char *msg);

// Launch KERNEL<B> (a kernel template over the workgroup size B; the _T form
// passes one more template argument, KERNEL<B, TARG>) with the table's B for
// `items` elements, one lane per element.
#define SUBDIV_LAUNCH_TUNED_T(key, items, stream, KERNEL, TARG, ...)                                          \
  do {                                                                                                        \
    const long long _n = (items);                                                                             \
    switch (tuned_block((key), _n)) {                                                                         \
      case 64:                                                                                                \
        hipLaunchKernelGGL(HIP_KERNEL_NAME(KERNEL<64, TARG>), dim3(grid_for(_n, 64)), dim3(64), 0, stream,     \
                           __VA_ARGS__);                                                                      \
        break;                                                                                                \
      case 128:                                                                                               \
        hipLaunchKernelGGL(HIP_KERNEL_NAME(KERNEL<128, TARG>), dim3(grid_for(_n, 128)), dim3(128), 0, stream,  \
                           __VA_ARGS__);                                                                      \
        break;                                                                                                \
      case 512:                                                                                               \
        hipLaunchKernelGGL(HIP_KERNEL_NAME(KERNEL<512, TARG>), dim3(grid_for(_n, 512)), dim3(512), 0, stream,  \
                           __VA_ARGS__);                                                                      \
        break;                                                                                                \
      default:                                                                                                \
        hipLaunchKernelGGL(HIP_KERNEL_NAME(KERNEL<256, TARG>), dim3(grid_for(_n, 256)), dim3(256), 0, stream,  \
                           __VA_ARGS__);                                                                      \
        break;                                                                                                \
    }                                                                                                         \
  } while (0)
#define SUBDIV_LAUNCH_TUNED(key, items, stream, KERNEL, ...)                                                        \
  do {                                                                                                              \
    const long long _n = (items);                                                                                   \
    switch (tuned_block((key), _n)) {                                                                               \
      case 64: hipLaunchKernelGGL(KERNEL<64>, dim3(grid_for(_n, 64)), dim3(64), 0, stream, __VA_ARGS__); break;     \
      case 128: hipLaunchKernelGGL(KERNEL<128>, dim3(grid_for(_n, 128)), dim3(128), 0, stream, __VA_ARGS__); break; \
      case 512: hipLaunchKernelGGL(KERNEL<512>, dim3(grid_for(_n, 512)), dim3(512), 0, stream, __VA_ARGS__); break; \
      default: hipLaunchKernelGGL(KERNEL<256>, dim3(grid_for(_n, 256)), dim3(256), 0, stream, __VA_ARGS__); break;  \
    }                                                                                                               \
  } while (0)

// ---- launchers (each returns hipGetLastError() of its launches) --------
hipError_t launch_fill_i32(int32_t *p, int32_t value, long long n, hipStream_t s);
// up to five int32 regions cleared to zero in one launch
struct ZeroRegions {
  int32_t *p[5];
  long long n[5];
  int count;
};
hipError_t launch_zero_regions(const ZeroRegions &z, hipStream_t s);
hipError_t launch_fill_u8(uint8_t *p, long long nbytes, hipStream_t s);
// channels c0..c0+2 of [V*dim] vertex data into a [V*3] array; up to six back
hipError_t launch_pack3(const float *data, int dim, int c0, long long V, float *slice, hipStream_t s);
hipError_t launch_unpack6(const float *a, const float *b, int dim, int c0, int ncols, long long V, float *out,
                          hipStream_t s);
// exclusive scan of n ints into out[0..n] (out[n] = total); partials needs scan_partials_ints(n) ints;
// when total_dst != nullptr the total is also stored there.
long long scan_partials_ints(long long n);
hipError_t launch_scan(const int32_t *in, int32_t *out, long long n, int32_t *partials, int32_t *total_dst,
                       hipStream_t s);

// Generic build (the symbolic pass + mapped M M^T of Sec. 4.2) on any level.
struct BuildScratch {
  int32_t *nval;     // [V+1]
  int32_t *rowptr;   // [V+1]
  int32_t *cursor;   // [V]
  int32_t *inc;      // [H]  half-edges leaving each vertex (row view of M)
  int32_t *cand;     // [2H] per-vertex candidate neighbour lists
  int32_t *cntlo;    // [V+1]
  int32_t *ebase;    // [V+1]
  int32_t *bflag;    // [H+1] boundary flag per edge id (E <= H)
  int32_t *sigcnt;   // [H]  crease tags per edge id
  int32_t *partials; // scan partials
};
// phase A: validation of faces / indices, valence counts, column of every
// non-zero (written to t.hface for a general cage)
// (cleared: the caller has zeroed b.nval [V+1] and b.cursor [V] already)
hipError_t build_faces(const Topo &t, int scheme, const BuildScratch &b, DeviceInfo *info, hipStream_t s,
                       bool cleared = false);
// phase B: row view of M, twins, edge ids, edge -> half-edge map, boundary flags
hipError_t build_adjacency(const Topo &t, int scheme, const BuildScratch &b, Adj &a, DeviceInfo *info,
                           hipStream_t s);
// counts the triangles of a triangle mesh whose three twins lie in one face
hipError_t count_pillows(const Topo &t, const Adj &a, DeviceInfo *info, hipStream_t s);
hipError_t build_creases(const Topo &t, const BuildScratch &b, const Adj &a, int num_creases,
                         const int32_t *crease_verts, const float *crease_sharp, DeviceInfo *info, hipStream_t s);
// boundary prefix of a built level (needs the DeviceInfo's E on device: passed as E)
hipError_t build_bscan(const Topo &t, const BuildScratch &b, Adj &a, hipStream_t s);
hipError_t launch_edge_export(const Topo &t, const Adj &a, int32_t *edge_out, hipStream_t s);

// Catmull-Clark level step.
struct CCStep {
  Topo t;
  Adj a;            // adjacency of level k (input)
  const float *P;   // [V*3]
  int32_t *fv1;     // [4H] refined M
  float *P1;        // [(V+F+E)*3]
  double *sig1;     // [E_{k+1}] inherited sharpness of level k+1 (null: not written)
  bool has_bnd;     // level k has boundary edges (bscan valid)
  bool creases;     // level k may have creases (a.sig, a.vcr valid)
  bool creases1;    // level k+1 may have creases
};
enum { CC_FACE = 0, CC_VERTEX = 1, CC_EDGE = 2 };
// one of the three kernels of a Catmull-Clark level (launch in this order)
hipError_t cc_launch(int which, const CCStep &c, hipStream_t s);

// Catmull-Clark level k >= 1 from the adjacency of its parent level m = k-1.
enum { LAG_GROUP = 0, LAG_VERTEX = 1, LAG_EDGE = 2 };
struct LagStep {
  Topo tm;              // parent level m
  Adj am;               // its adjacency (twin, eid, vhe, e2h, bscan; E = E_m)
  bool bnd;             // the mesh has boundary edges (bscan valid)
  int32_t Vk, Fk, Ek;   // sizes of level k
  const float *Pk;      // [Vk*3]
  const double *sigk;   // [Ek] crease sharpness of level k, or nullptr
  int4 *vcrk;           // [Vm] crease valency / first two creases of level-m vertices at level k
  float *P1;            // [(Vk+Fk+Ek)*3] positions of level k+1
  int32_t *fv1;         // [16*Hm] mesh matrix of level k+1, or nullptr
  int32_t *fvk;         // [4*Hm] mesh matrix of level k, or nullptr
  double *sig1;         // [E_{k+1}] sharpness of level k+1, or nullptr
  int32_t *edges_k;     // [2*Ek] (lo, hi) of level-k edges, or nullptr
  Adj ak;               // level-k adjacency to emit (twin/eid/vhe/e2h/bscan), nullptrs = none
};
hipError_t lag_launch(int which, const LagStep &c, hipStream_t s);

// Crease-free Catmull-Clark level k >= 3: the parent m = k-1 and grandparent
// g = k-2 are quad levels, so each level-m vertex's ring is known from the
// corner it occupies in its level-m faces (see cc_lag.hip).
enum { LAG2_GROUP = 0, LAG2_COMBINE = 1, LAG2_OLDER = 2 };
struct Lag2Step {
  LagStep s;                 // the parent-level view (creases: s.sigk, s.vcrk)
  int32_t Vg, Fg, Eg, VFg;   // grandparent sizes, VFg = Vg + Fg
  int32_t Vq, Fq;            // sizes of the level below g when it is all quads (else 0): the
                             // level-g vertices [Vq, Vq+Fq) are its face points, the rest its edge points
  const int32_t *vhe_g;      // grandparent adjacency
  const int32_t *twin_g;
  const int32_t *e2h_g;
  const int32_t *bscan_g;    // grandparent boundary-edge prefix (meshes with boundary)
  float *hs;                 // [2*Eg*3] half rings of the grandparent's edge points
  float *term0;              // [Fm*3] ring term of corner 0 of every level-m face
};
hipError_t lag2_launch(int which, const Lag2Step &c, hipStream_t s);

// Adjoint of one Catmull-Clark level: g0 = R_k^T g1 (launch in this order).
enum { BW_COEF = 0, BW_FACE = 1, BW_VERTEX = 2 };
struct BwdStep {
  Topo t;            // level k
  Adj a;             // its adjacency (twin, eid, vhe; sig when the level may carry creases)
  const float *g1;   // [V_{k+1}*3] gradient w.r.t. the positions of level k+1
  float *g0;         // [V_k*3] gradient w.r.t. the positions of level k
  float *term;       // [H_k*3] scratch: each half-edge's share of its origin's gradient
  float *coef;       // [V_k*4] scratch: vertex-rule coefficients (a, b, d, flags)
  // levels k >= 2 (refined from a quad level k-1): the sizes of level k-1,
  // whose face and edge points are the level-k vertices [Vp, Vp+Fp) and
  // [Vp+Fp, V_k), and its boundary prefix (nullptr without a boundary);
  // Vp = 0 on the levels below
  int32_t Vp, Fp;
  const int32_t *bscan_p;
};
hipError_t bw_launch(int which, const BwdStep &c, hipStream_t s);

// ---- selective subdivision: extraction of a region of a cage ------------
struct SelectScratch {
  int32_t *x[2];               // [V] vertex flags, alternating over the rings (the last in x[rings & 1])
  int32_t *q;                  // [F] face flags
  int32_t *vnew, *fnew, *onew; // [V+1], [F+1], [F+1] exclusive scans: new vertex / face ids, corner offsets
  int32_t *flag;               // [max(F, H)+1] corner counts of a general cage, then crease flags
  int32_t *cnew;               // [H+1] crease ids
  int32_t *partials;           // scan partials (max(V, H) items)
  int32_t *totals;             // [4] V', F', H' (general cages), C'
  uint8_t *seed0;              // [V] the seed flags x_0
  int32_t *qadd;               // [F] faces added by the pinch passes
  int32_t *changed;            // [kPinchPasses] 1 when that pass added faces
};
// passes of the pinch closing of a selection (SUBDIV_SELECT_CLOSE_PINCHES)
constexpr int kPinchPasses = 16;
struct ExtractOut {
  uint8_t *seed;               // [V'] x_0 of every extracted vertex, or nullptr
  int32_t *fv, *off, *fmap, *vmap, *cv;
  float *P, *cs;
  int32_t F, C;
};
// flags and scans; totals are left on the device for one read-back
// close_pinches: after the rings, every selected vertex whose selected faces
// form more than one fan gets its whole star selected, pass after pass, until
// no such vertex is left (at most kPinchPasses passes; changed[] tells)
hipError_t select_region(const Topo &t, const Adj &a, const SelectScratch &w, const uint8_t *seed,
                         const int32_t *valence, int rings, bool close_pinches, hipStream_t s);
hipError_t extract_region(const Topo &t, const Adj &a, const SelectScratch &w, int rings, const float *P,
                          const ExtractOut &o, hipStream_t s);

// ---- batches: meshes packed into one disjoint union cage ---------------
struct BatchMesh {        // one mesh of a batch (device table entry)
  const int32_t *fv;
  const int32_t *off;     // nullptr for a uniform face order
  int32_t order;
  const float *P;
  const int32_t *cv;
  const float *cs;
  int32_t V, F, H, C;
  int32_t vofs, fofs, hofs, cofs;  // its first vertex / face / half-edge / crease in the union
};
struct BatchUnion {       // the union cage's buffers
  int32_t *fv;
  int32_t *off;           // nullptr when the union has a uniform order
  int32_t *cv;
  float *cs;
};
// Gather of the union's final level L into the meshes' own buffers. The
// union's level-L vertex ids are blocks [V_0 | F_0 | E_0 | F_1 | E_1 | ...]
// (Catmull-Clark; Loop has no F blocks, sqrt(3) no E blocks), every block
// listing the meshes in order; mesh i numbers its own level-L vertices by its
// segments of the same blocks, in the same block order.
constexpr int kGather = 1024;  // elements per workgroup of the gather kernels
struct BatchTables {
  int32_t n, order, nblk, nseg;  // meshes, face order, blocks, segments (nblk * n)
  const int4 *seg;       // [nseg] (union start, mesh, local start, length), in union order
  const int32_t *pch;    // [nseg+1] chunk prefix of the segments (kGather vertices per chunk)
  const int32_t *ub;     // [nblk+1] union start of every block
  const int32_t *doff;   // [nblk*n] local id - union id inside segment (block b, mesh i)
  const int32_t *fpre;   // [n+1] union face prefix of level L
  const int32_t *fch;    // [n+1] chunk prefix of the meshes' faces (kGather faces per chunk)
};
struct BatchOut {
  int32_t *fv;
  float *P;
};
hipError_t batch_concat_topology(const BatchMesh *m, int n, const BatchUnion &u, long long items, hipStream_t s);
hipError_t batch_concat_positions(const BatchMesh *m, int n, float *P, long long V, hipStream_t s);
// per-mesh edge prefix [n+1], boundary edges, largest valence and largest
// crease sharpness (float bits) [n] each; bcount, vmax, smax consecutive
hipError_t batch_stats(const BatchMesh *m, int n, const int32_t *ebase, const int32_t *bflag, const int32_t *rowptr,
                       const float *cs, long long VU, long long HU, long long CU, int32_t *epre, int32_t *bcount,
                       int32_t *vmax, int32_t *smax, hipStream_t s);
hipError_t batch_extract(const BatchTables &t, const int32_t *fvL, const float *PL, const BatchOut *out,
                         int face_chunks, int vertex_chunks, hipStream_t s);

// Loop / sqrt(3) level steps. `a` is the adjacency of level k (from the
// build of the cage, or carried over from the previous step). When level
// k+1 is refined further, the step also writes level k+1's adjacency in
// closed form into `a1` (twin, eid, e2h, vhe); `base` holds the edge bases of
// level k+1's edges grouped by their higher end (counts, then their scan).
struct TriStep {
  Topo t;
  Adj a;
  const float *P;
  int32_t *fv1;
  float *P1;
  Adj a1;
  int32_t *base;
  int32_t nbnd;  // boundary edges of level k (sqrt(3): they keep ids 0 .. nbnd-1 on level k+1)
  int32_t Vg;    // levels >= 1: vertices of the level k was refined from (its old vertices); 0 on the cage
  Adj ap;        // levels >= 1: adjacency of that level (twin, eid, vhe), where the old vertices' rings are walked
  int32_t Vq;    // levels >= 2: vertices of level k-2 (the old vertices v >= Vq are its edge / face points)
  Adj app;       // when set (twin != nullptr): adjacency of level k-2, where the rings of v < Vq are walked
  int32_t Vr;    // with app: vertices of level k-3 (0 when level k-2 is the cage)
  // sqrt(3), when set (a0.twin != nullptr): the cage's adjacency, from which the
  // rings of the cage vertices and of the cage's face points are read instead
  Adj a0;
  int32_t V0, F0;  // the cage's vertices and faces
  int32_t pow3;    // 3^(l-1), l >= 1 the level whose face points are the neighbours (Vg = V_l)
  // rings walked on level k itself (Vg = 0) of a refined level: the points
  // fpV .. fpV + fpF - 1 born from the faces of level k-1 (fpF = 0: none)
  int32_t fpV, fpF;
  // level k made by a trisection step (sqrt(3) with the boundary cycle): the
  // boundary slot and rank of each level-(k-1) face (with ap = level k-1's
  // adjacency), from which the old vertices' rings follow; nullptr otherwise
  const int32_t *pbslot, *pbrank;
  // sqrt(3), last step from two levels down: the points Vq .. Vg - 1 (face
  // points of level k-2) whose three edges are interior already have theirs
  int32_t fp_done;
};
enum { LOOP_EDGE = 0, LOOP_VERTEX = 1, LOOP_FACE = 2, SQRT3_FACE = 3, SQRT3_VERTEX = 4, SQRT3_COUNT = 5 };
hipError_t tri_launch(int which, const TriStep &c, hipStream_t s);
// Loop creases of level k (c.a.sig, c.a.vcr): crease and corner vertices over
// the smooth vertex points, then (sig1 != nullptr, with c.base) the
// inherited sharpness of level k+1's edges into sig1 (cleared by the caller)
hipError_t loop_crease_launch(const TriStep &c, double *sig1, hipStream_t s);

// Trisection step of sqrt(3) with Kobbelt's boundary cycle (see tri.hip):
// level k (whose faces have at most one boundary edge each) to level k+1.
struct TrisectStep {
  Topo t;
  Adj a;            // level k: twin, vhe (the boundary half-edge of a boundary vertex)
  const float *P;
  int32_t *fv1;     // [9 F] children
  float *P1;        // [(V + F + B) * 3]
  int32_t *bslot;   // [F] slot of the face's boundary edge, or -1
  int32_t *brank;   // [F + 1] boundary flags, scanned into the ranks among the boundary faces
  int32_t *bnb;     // [2 V] previous and next boundary neighbour of a boundary vertex
  // carried adjacency of level k+1 (a1.twin null: none)
  Adj a1;           // twin, eid [9 F], vhe [V + F + B], e2h, bscan (boundary edges only) [E']
  int32_t *base;    // [2 F + 1] edge counts per higher end (points p / face points, then q), scanned
  uint8_t *pmask;   // [F] bit i: the point across edge i toward this face is a face point or p
  int32_t nbnd;     // B = boundary faces of level k
  int32_t fpV, fpF; // level k's face points of the faces of level k-1 (fpF = 0 on the cage)
  Adj ap;           // optional (twin != nullptr): level k-1's adjacency, where the old vertices'
                    // rings are walked (level k came from it by a sqrt(3) step)
};
enum { TRISECT_MARK = 0, TRISECT_FACE = 1, TRISECT_VERTEX = 2, TRISECT_COUNT = 3 };
hipError_t trisect_launch(int which, const TrisectStep &c, hipStream_t s);

// Last Loop or sqrt(3) step k -> k+1 computed from level m = k-1 (which
// level k was refined from): its faces, edges and adjacency are a quarter
// (a third) the size of level k's, and level k's are closed-form functions of
// them, so level k's adjacency is never written.
struct TriLag {
  Topo tm;               // level m (triangles)
  Adj am;                // level m: twin, eid, e2h (E = |e_m|)
  const int32_t *base;   // Loop: [E_m + 1] first level-k edge id with higher end EP(e), per level-m edge;
                         // sqrt(3), with edges: [F_m + 1] first id (after the boundary ones) with higher end F_r
  const float *Pk;       // level-k positions [V_k]
  int32_t Vk;            // V_k = V_m + E_m (Loop), V_m + F_m (sqrt(3))
  int32_t Ek;            // Loop: E_k = base[E_m]
  int32_t *fv2;          // level k+1 face table (Loop [48 F_m], sqrt(3) [27 F_m])
  float *P2;             // level k+1 positions [V_{k+1}]
  int32_t *edges;        // optional: (lo, hi) of level k's edges in id order [2 E_k]
  int32_t Bk;            // sqrt(3): boundary edges of level k (its first ids)
  int32_t *cnt1;         // Loop, optional: [E_k] per level-k edge 2 + |N(e) below e| (scanned
                         // afterwards into level k's own edge bases)
  float *Pk2;            // optional: level k+2 positions; the lane also writes the level-(k+2)
                         // point of its level-k point (Loop: E_e; sqrt(3): F_r, when r's edges
                         // are interior), whose level-(k+1) ring the lane holds
  const int32_t *vhek;   // with Pk2: level k's ring starts (the start picks the ring's order)
};
enum { LAG_LOOP_FACE = 0, LAG_LOOP_EDGE = 1, LAG_SQRT3_FACE = 2 };
hipError_t tri_lag_launch(int which, const TriLag &c, hipStream_t s);
hipError_t init_weight_tables();

}  // namespace subdiv
