/*
 * subdiv.h - C ABI of the MI355X (gfx950) AlSub refinement library.
 *
 * One call refines a polygon control mesh L levels with Catmull-Clark, Loop
 * or sqrt(3) subdivision, written as the sparse-matrix algebra of AlSub
 * (Mlakar et al., "AlSub: Fully Parallel and Modular Subdivision", ACM TOG):
 *
 *   - the mesh is its mesh matrix M (Sec. 3.2): one column per face, row
 *     indices = the face's vertices in counter-clockwise cyclic order;
 *     a uniform face order drops the column pointer (reduced form, Sec. 4.1);
 *   - a build step derives edge ids (the upper triangle of E = M M^T mapped
 *     with Q_c + Q_c^{c-1}, eq:CC_E) and face adjacency (F = M M^T mapped with
 *     Q_c, eq:F; G for Loop, App. B) and emits the refined mesh matrix
 *     (Sec. 3.2 "Topology refinement", App. A, App. B);
 *   - an eval step computes face, edge and vertex points (eq:spla_fp, the
 *     edge-point rule, eq:vo and the vertex update; equ:sqrt2; eq:loop_smooth),
 *     boundary repair (eq::CC_boundary) and creases (Sec. 3.3).
 *
 * All pointers in these structs are DEVICE pointers owned by the caller.
 * The library never allocates device memory in these calls: every buffer is
 * the caller's (outputs) or carved from the caller's workspace. All work is
 * enqueued on the given HIP stream (`void *stream` is a hipStream_t, NULL =
 * the null stream). Calls on different streams with different workspaces are
 * independent; calls sharing a workspace must be serialised by the caller.
 *
 * Vertex order of a refined level (fixed by the paper's index rules):
 *   Catmull-Clark  [vertex points | face points | edge points]  (|v|+r, |v|+|f|+e)
 *   Loop           [vertex points | edge points]
 *   sqrt(3)        [vertex points | face points]                (App. A, |v|+i)
 *   trisection     [vertex points | face points or p | q]       (SUBDIV_SQRT3_KOBBELT, even levels)
 * Edge ids enumerate the strict upper triangle of E in CSC order, i.e. the
 * edges {lo < hi} sorted ascending by (hi, lo).
 * Child faces: Catmull-Clark child j of face r is at col_ptr[r] + j and is
 * (v_j, edge(v_j,v_j+1), face r, edge(v_j-1,v_j)); Loop children 4r+j (j<3)
 * are (v_j, e(j,j+1), e(j-1,j)) and 4r+3 = (e01, e12, e20); sqrt(3) child
 * 3r+j is (v_j, face across edge j, face r), or (v_j, v_j+1, face r) on a
 * boundary edge.
 */
#ifndef SUBDIV_H
#define SUBDIV_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

/* ---- schemes and status codes ---------------------------------------- */
enum {
  SUBDIV_CATMULL_CLARK = 0, /* Sec. 3 */
  SUBDIV_LOOP = 1,          /* App. B, triangle meshes */
  SUBDIV_SQRT3 = 2,         /* App. A, triangle meshes; boundary vertices fixed, boundary edges kept */
  SUBDIV_SQRT3_KOBBELT = 3  /* App. A with the boundary rule it defers to Kobbelt's sqrt(3) paper: a two-step
                               cycle, levels 1, 3, ... by the sqrt(3) step with the boundary fixed, levels 2,
                               4, ... by a trisection step that splits every boundary edge in three (a boundary
                               face r gets two edge points instead of its face point: p at |v| + r, q at
                               |v| + |f| + its rank among the boundary faces) with the ternary cubic B-spline
                               rule on the boundary. Triangle meshes, no creases; both steps carry the next
                               level's adjacency over in closed form (the generic mapped product on request, as
                               for the other schemes); not in batches, no kept state */
};

enum {
  SUBDIV_OK = 0,
  SUBDIV_INVALID_ARG = -1,  /* null or misaligned pointer, bad enum/level count, index out of range, size overflow */
  SUBDIV_SCHEME_MESH = -2,  /* Loop / sqrt(3) given a face that is not a triangle */
  SUBDIV_NONMANIFOLD = -3,  /* edge with > 2 faces, a directed edge twice, a vertex whose faces form > 1 fan,
                               or (Loop / sqrt(3), levels > 1) two triangles on the same three vertices, whose
                               first refined level has edges on four faces */
  SUBDIV_DEGENERATE = -4,   /* face order < 3, repeated vertex in a face, or a vertex in no face */
  SUBDIV_BAD_CREASE = -5,   /* crease end points not an edge, sharpness < 0 or NaN, or an edge tagged twice */
  SUBDIV_WORKSPACE = -6,    /* workspace too small */
  SUBDIV_HIP = -7,          /* a HIP runtime call failed; subdiv_last_error() has the HIP message */
  SUBDIV_STATE = -8         /* plan / state does not match the call (different mesh or scheme) */
};

/* When an input has several faults, the code reported is the first of
 * INVALID_ARG, SCHEME_MESH, DEGENERATE, NONMANIFOLD, BAD_CREASE that applies. */

#define SUBDIV_MAX_LEVELS 10
#define SUBDIV_MAX_VALENCE 1024 /* vertices of higher valence are rejected (INVALID_ARG) */

/* flags for subdiv_plan */
#define SUBDIV_FLAG_REBUILD_EACH_LEVEL 1u /* rebuild E/F from M at every level (generic M M^T path)
                                             instead of carrying them over in closed form */
#define SUBDIV_FLAG_KEEP_STATE 2u         /* keep every level's topology in the workspace for
                                             subdiv_refine_positions, subdiv_refine_vertex_data
                                             (every scheme but SUBDIV_SQRT3_KOBBELT) and
                                             subdiv_backward (Catmull-Clark;
                                             its first call after a subdiv_refine also writes the
                                             adjoint's per-vertex rule coefficients there); not
                                             with SUBDIV_FLAG_REBUILD_EACH_LEVEL */

/* ---- inputs ----------------------------------------------------------- */
typedef struct subdiv_mesh {
  int32_t num_vertices;           /* |v| >= 1 */
  int32_t num_faces;              /* |f| >= 1 */
  int32_t face_order;             /* 3 or 4 when face_offsets == NULL (reduced M), else ignored */
  int32_t num_halfedges;          /* H = nnz(M); must equal face_offsets[|f|] when face_offsets != NULL,
                                     ignored (= |f|*face_order) otherwise */
  const int32_t *face_offsets;    /* [|f|+1] column pointer of M (starts at 0, non-decreasing), or NULL */
  const int32_t *face_verts;      /* [H] row indices of M, CCW per face; 16-byte aligned */
  const float *positions;         /* [|v|*3] row-major x,y,z */
  int32_t num_creases;            /* crease matrix C as a list (Sec. 3.3); Catmull-Clark and Loop
                                     (Loop takes the same crease rules on its own points);
                                     sqrt(3) returns SUBDIV_INVALID_ARG */
  const int32_t *crease_verts;    /* [2*num_creases] end points of crease edges */
  const float *crease_sharpness;  /* [num_creases] sharpness sigma >= 0 (0 = smooth edge) */
} subdiv_mesh;

/* ---- sizes ------------------------------------------------------------ */
typedef struct subdiv_level_info {
  int64_t num_vertices;
  int64_t num_edges;
  int64_t num_faces;
  int64_t num_halfedges;     /* H = nnz(M) */
  int64_t num_boundary_edges;
  int32_t face_order;        /* uniform face order, 0 = mixed (column pointer present) */
  int32_t max_creases;       /* upper bound on the crease edges of this level (0 = smooth) */
} subdiv_level_info;

typedef struct subdiv_plan_info {
  int32_t scheme;
  int32_t levels;
  uint32_t flags;
  int32_t max_valence;
  float max_sharpness;
  int32_t reserved0;
  subdiv_level_info level[SUBDIV_MAX_LEVELS + 1]; /* level[0] = the cage */
  size_t workspace_bytes;   /* device workspace subdiv_refine needs */
  /* private to the library: identity of the cage and of the plan workspace */
  const void *priv_mesh_verts;
  const void *priv_ws;
  uint64_t priv_stamp;
} subdiv_plan_info;

/* ---- outputs ---------------------------------------------------------- */
/* One refined level, all device buffers owned by the caller. face_verts has
 * level[k].num_halfedges entries (F*4 for Catmull-Clark, F*3 for Loop and
 * sqrt(3)); positions has level[k].num_vertices*3 floats. Optional buffers
 * may be NULL. */
typedef struct subdiv_level_out {
  int32_t *face_verts;       /* [H_k] reduced M of level k (uniform order); 16-byte aligned */
  float *positions;          /* [V_k*3] */
  int32_t *edge_verts;       /* optional [2*E_{k-1}]: (lo, hi) of the PARENT level's edges in id order */
  double *crease_sharpness;  /* optional [E_k]: sharpness per edge id of level k (0 = smooth);
                                written only while max_creases > 0 */
} subdiv_level_out;

/* Upper bound of the workspace bytes subdiv_plan and subdiv_refine need for
 * a cage of V vertices, F faces, H = nnz(M) and C creases refined `levels`
 * times (host-only, no device work). A workspace of this size can be passed
 * to subdiv_plan and then, unchanged, to subdiv_refine, which then reuses the
 * plan's level-0 adjacency instead of rebuilding it. */
size_t subdiv_workspace_bound(int32_t V, int32_t F, int64_t H, int32_t C, int scheme, int levels, uint32_t flags);

/* Symbolic pass (Sec. 4.2): validates the cage, builds its edge ids and
 * adjacency on the device in `ws`, waits for the stream, and fills `plan`
 * with the exact size of every level and the workspace subdiv_refine needs.
 * Returns SUBDIV_OK or a status code; on error `plan` is zeroed. */
int subdiv_plan(const subdiv_mesh *mesh, int scheme, int levels, uint32_t flags, void *ws, size_t ws_bytes,
                subdiv_plan_info *plan, void *stream);

/* Refines the cage plan->levels times (dynamic topology: build and eval
 * alternate per level, Sec. 3.6). outs[k] for k = 1..levels receive level k;
 * outs[levels].face_verts and .positions are required, the other levels are
 * written only where the caller gives buffers (outs may hold NULLs there;
 * outs[0] is ignored). `ws` needs plan->workspace_bytes bytes; when it is the
 * workspace plan used, the level-0 adjacency is reused. The mesh must be the
 * one planned (same face_verts pointer); positions may change, the crease
 * tags and sharpness are read by subdiv_plan.
 * Output buffers of different levels must not overlap, with one exception:
 * level levels-2's positions may share the final positions' buffer (it is
 * not read after the final level's first write). For Loop and sqrt(3) the
 * step before the last writes part of the final positions early, and skips
 * that when the final positions overlap level levels-2's or levels-1's.
 * Enqueues work only: no host synchronisation. */
int subdiv_refine(const subdiv_mesh *mesh, const subdiv_plan_info *plan, subdiv_level_out *outs, void *ws,
                  size_t ws_bytes, void *stream);

/* ---- refinement in the library's own workspace -------------------------
 * For callers that cannot allocate device memory at all (code under HIP
 * graph capture, tight serving loops, harnesses that forbid hipMalloc):
 * subdiv_refine with the workspace taken from a device array the library
 * holds for the life of the process, SUBDIV_STATIC_WORKSPACE_BYTES on every
 * GPU it runs on (each device has its own copy; its address is looked up
 * once per device, on the first call with that device current). The call
 * allocates nothing: no hipMalloc, hipFree or allocating library routine.
 * The caller still passes the mesh, a plan from subdiv_plan (made with any
 * workspace; the cage adjacency is built again in the library's workspace
 * unless the previous call on this device refined the same plan) and the
 * outputs, as for subdiv_refine. Every call on a GPU shares that GPU's array,
 * which keeps the last call's contents: calls that overlap on one GPU (other
 * streams, other threads) race and must be serialised by the caller.
 * Returns SUBDIV_WORKSPACE when plan->workspace_bytes exceeds the array
 * (subdiv_last_error() then names both sizes), SUBDIV_INVALID_ARG for a plan
 * made with SUBDIV_FLAG_KEEP_STATE (its state would live in memory the
 * caller cannot pass to subdiv_backward), and otherwise what subdiv_refine
 * returns. Enqueues work only. */
#define SUBDIV_STATIC_WORKSPACE_BYTES ((size_t)64 << 20)
int subdiv_refine_static(const subdiv_mesh *mesh, const subdiv_plan_info *plan, subdiv_level_out *outs,
                         void *stream);

/* Adjoint of the refinement (reverse mode; Catmull-Clark). Refinement is
 * linear in the vertex data, P_L = R P_0 with R = R_{L-1} ... R_0 fixed by
 * the topology and creases (Sec. 3.6, eq:singleSpMV), so
 * grad_in = R^T grad_out, computed level by level as transposed gathers over
 * the adjacency each level kept. Requires a plan made with
 * SUBDIV_FLAG_KEEP_STATE and a completed subdiv_refine with the same plan,
 * mesh and workspace (the workspace holds every level's topology; it must not
 * be reused in between). grad_out: [V_L*3] device, grad_in: [V_0*3] device,
 * both caller-owned; grad_in is overwritten. Enqueues work only.
 * Returns SUBDIV_STATE when the plan was not made for the adjoint (no
 * SUBDIV_FLAG_KEEP_STATE, or a Loop or sqrt(3) plan), or when no
 * subdiv_refine with this plan has been enqueued into `ws` since the last
 * subdiv_plan, batch plan or subdiv_state_destroy that touched it (the
 * library keeps a host-side record per workspace; it never reads state that
 * was not written). */
int subdiv_backward(const subdiv_mesh *mesh, const subdiv_plan_info *plan, const float *grad_out, float *grad_in,
                    void *ws, size_t ws_bytes, void *stream);

/* The state of a refinement is the pair (plan, workspace): the plan holds
 * the sizes, the caller's workspace the level-0 adjacency (after subdiv_plan
 * or subdiv_refine) and, with SUBDIV_FLAG_KEEP_STATE, every level's topology
 * and the adjoint's coefficients (after subdiv_refine). The library keeps a
 * small host-side record of which plan each workspace holds; this call drops
 * the record of `ws` when it belongs to `plan`, so that later calls that
 * need the state (subdiv_backward, subdiv_refine_positions,
 * subdiv_refine_vertex_data, subdiv_select, subdiv_extract) return
 * SUBDIV_STATE and subdiv_refine rebuilds the cage adjacency. The device
 * memory stays the caller's: free or reuse it once the work enqueued on it
 * has completed. Host-only, no device work. Returns SUBDIV_STATE when `ws`
 * holds no state of `plan`, SUBDIV_INVALID_ARG for null pointers. */
int subdiv_state_destroy(const subdiv_plan_info *plan, const void *ws);

/* ---- mesh reordering (Sec. 4.5) --------------------------------------------
 * Reverse Cuthill-McKee on the cage's vertex graph, for locality of the rows
 * and columns of M in memory. HOST pointers: face_offsets ([F+1], or NULL
 * for a uniform face_order) and face_verts ([H]) as in subdiv_mesh;
 * vertex_perm [V] and face_perm [F] receive new id -> old id. Each connected
 * component starts at its unvisited vertex of smallest degree (distinct
 * neighbours; smaller id first), a dequeued vertex appends its unvisited
 * neighbours by increasing (degree, id), and the sequence is reversed. Faces
 * are ordered by the smallest new id among their corners (their first
 * non-zero), then by old id; applying the permutations (corners renumbered,
 * cyclic order kept) is the caller's. Runs on the host, synchronously.
 * Returns SUBDIV_INVALID_ARG for sizes, pointers or indices out of range. */
int subdiv_rcm_order(int32_t num_vertices, int32_t num_faces, const int32_t *face_offsets, int32_t face_order,
                     const int32_t *face_verts, int32_t *vertex_perm, int32_t *face_perm);

/* ---- selective subdivision: extraction of a region (Sec. 3.4) ----------
 * x_0 marks the seed vertices; q_i = M^T x_i marks the faces with a marked
 * corner and x_{i+1} = M q_i their corners, for i < rings. The extraction
 * M' = X M X-ring keeps the faces of q_{rings-1} and the vertices of x_rings
 * (the identity with unselected rows / columns deleted), P' = X P. Survivors
 * keep their relative order: the extracted vertex of rank r is the r-th
 * selected cage vertex, faces keep their corners in cyclic order. Creases
 * whose edge is an edge of an extracted face are kept (endpoints renumbered,
 * same sharpness); the rest are dropped. The extraction is a cage like any
 * other: plan and refine it with its own workspace.
 * Both calls need the cage's successful subdiv_plan (any scheme) with the
 * same mesh and workspace, whose level-0 region holds the selection between
 * the two calls (a later subdiv_plan into the workspace replaces it). */
typedef struct subdiv_selection {
  int32_t num_vertices;   /* V' of the extraction (0: nothing selected) */
  int32_t num_faces;      /* F' */
  int32_t num_halfedges;  /* H' */
  int32_t num_creases;    /* C' */
  int32_t face_order;     /* the cage's uniform order (3 or 4), or 0: the extraction has a column pointer */
  int32_t rings;
  uint32_t flags;         /* the selection's flags (subdiv_select_ex) */
  uint64_t priv_stamp;    /* private: the plan it was made with */
  const void *priv_ws;
} subdiv_selection;

/* Caller-allocated device buffers of the extraction, sized from a selection. */
typedef struct subdiv_extraction {
  int32_t *face_offsets;     /* [F'+1] when face_order == 0, else unused */
  int32_t *face_verts;       /* [H'] extracted vertex ids */
  float *positions;          /* [V'*3] copies of the selected cage positions */
  int32_t *crease_verts;     /* [2*C'] (may be NULL when C' = 0) */
  float *crease_sharpness;   /* [C'] */
  int32_t *vertex_map;       /* [V'] cage id of every extracted vertex, or NULL */
  int32_t *face_map;         /* [F'] cage id of every extracted face, or NULL */
  uint8_t *seed_flags;       /* [V'] x_0 of every extracted vertex (1: it was a seed), or NULL: the
                                seeds carried into the extraction, for feature-adaptive refinement
                                that selects and extracts again on every refined level */
} subdiv_extraction;

/* Selection: seed is a [V] device byte mask (non-zero = selected) or NULL for
 * the extraordinary vertices, those whose valence n = M 1 (eq:vo: incident
 * faces) is not 4 (on an open cage this includes the boundary). rings >= 1.
 * Reads back the extraction's sizes into *sel (one synchronisation of the
 * stream). Returns SUBDIV_STATE without the cage's plan in this workspace. */
int subdiv_select(const subdiv_mesh *mesh, const subdiv_plan_info *plan, const uint8_t *seed, int rings, void *ws,
                  size_t ws_bytes, subdiv_selection *sel, void *stream);

/* The selection with options. SUBDIV_SELECT_CLOSE_PINCHES: after the rings,
 * every selected vertex whose selected faces form more than one fan around
 * it (two selected regions touching at one vertex, which would make the
 * extraction non-manifold there) gets its whole star selected, and the pass
 * repeats until no such vertex is left (every pass reads the previous pass's
 * selection only, so the result does not depend on thread order); a
 * selection still pinched after 16 passes returns SUBDIV_NONMANIFOLD. This is
 * the selection of feature-adaptive refinement, which extracts again on every
 * refined level. flags 0 is subdiv_select. */
#define SUBDIV_SELECT_CLOSE_PINCHES 1u
int subdiv_select_ex(const subdiv_mesh *mesh, const subdiv_plan_info *plan, const uint8_t *seed, int rings,
                     uint32_t flags, void *ws, size_t ws_bytes, subdiv_selection *sel, void *stream);

/* Extraction into the caller's buffers; enqueues work only. An empty
 * selection writes nothing. Returns SUBDIV_STATE when sel was not made with
 * this plan and workspace, SUBDIV_INVALID_ARG for a missing buffer. */
int subdiv_extract(const subdiv_mesh *mesh, const subdiv_plan_info *plan, const subdiv_selection *sel,
                   const subdiv_extraction *out, void *ws, size_t ws_bytes, void *stream);

/* Static topology (Sec. 3.6: P_L = R_{L-1} ... R_0 P_0 with every R_k fixed
 * by topology and creases). Re-evaluates the positions of a refinement (any
 * scheme) planned with SUBDIV_FLAG_KEEP_STATE, after one completed
 * subdiv_refine with the same plan, cage topology and workspace, for the
 * cage positions now in mesh->positions. The operators are applied
 * matrix-free by the same stencil kernels as subdiv_refine, reading the kept
 * face tables, adjacency and sharpness; nothing but positions is written, so
 * the result equals subdiv_refine's positions bit for bit. outs[k].positions
 * as in subdiv_refine (the final level is required; other fields are
 * ignored). Enqueues work only. Returns SUBDIV_STATE for a plan that does not
 * keep its state, or a workspace into which no subdiv_refine with this plan
 * was enqueued (see subdiv_backward). */
int subdiv_refine_positions(const subdiv_mesh *mesh, const subdiv_plan_info *plan, subdiv_level_out *outs, void *ws,
                            size_t ws_bytes, void *stream);

/* General vertex data: UVs, colours, any number of channels (Sec. 3.6:
 * refinement is linear in the vertex data and every channel goes through the
 * same R_{L-1} ... R_0, fixed by topology and creases). Refines data
 * ([V_0*dim] device floats, row-major: vertex v's channels at v*dim) into
 * out ([V_L*dim] device floats, caller-owned, overwritten), dim >= 1. The
 * state requirements are those of subdiv_refine_positions (a plan of any
 * scheme with SUBDIV_FLAG_KEEP_STATE, one completed subdiv_refine with the
 * same plan, cage topology and workspace). Channels go three at a time through
 * the kernels of subdiv_refine_positions: channels 3c..3c+2 of out equal, bit
 * for bit, the positions it writes for those three channels as cage
 * positions (channels past dim read as zero). Between calls the workspace
 * holds nothing of the data (the slices use the adjoint's scratch, so a
 * pending subdiv_backward on the same workspace must be ordered before).
 * Enqueues work only. Returns SUBDIV_INVALID_ARG for dim < 1 or a null
 * pointer, SUBDIV_STATE as subdiv_refine_positions. */
int subdiv_refine_vertex_data(const subdiv_mesh *mesh, const subdiv_plan_info *plan, const float *data, int dim,
                              float *out, void *ws, size_t ws_bytes, void *stream);

/* ---- batches of uneven meshes -----------------------------------------
 * A batch lists n meshes, each with its own scheme and level count. The
 * meshes are grouped by (scheme, levels), in order of first appearance; the
 * members of a group are packed into one disjoint union cage and refined
 * together, every stage one launch over the whole group, and a group of one
 * is refined as the mesh itself. Each mesh's final level is written to its
 * own buffers in its own numbering and is bit-identical to refining that mesh
 * alone (the union's index rules keep every mesh's elements in their
 * relative order). Loop and sqrt(3) need triangle meshes; creases in batches:
 * Catmull-Clark only.
 *
 * The refinement reads each mesh's counts (edges, boundary edges, largest
 * sharpness) from a plan of that mesh - made by subdiv_plan, or for a whole
 * batch at once by subdiv_plan_batch - so subdiv_refine_batch never waits for
 * the device: a server that keeps the plans of the cages it has seen enqueues
 * a whole batch without a host round trip. */
#define SUBDIV_MAX_BATCH 65536

/* Workspace bytes a batch needs (host-only): the larger of what
 * subdiv_plan_batch and subdiv_refine_batch use. With plans (one per mesh,
 * as subdiv_refine_batch takes them) the refinement's part is exact;
 * plans == NULL gives an upper bound from the sizes alone. `meshes` are read
 * for their sizes only. Returns 0 for invalid arguments or plans that do not
 * match their meshes. */
size_t subdiv_batch_workspace_bound(const subdiv_mesh *meshes, const int *schemes, const int *levels, int n,
                                    const subdiv_plan_info *plans, uint32_t flags);

/* Symbolic pass of a whole batch (Sec. 4.2, per group of the batch):
 * validates every mesh, builds each group's union adjacency, reads back all
 * counts and faults in one synchronisation of the stream, and fills
 * plans[i] with the sizes of every level of mesh i for levels[i] levels.
 * Each plans[i] is a plan of mesh i like subdiv_plan's (it can be passed to
 * subdiv_refine with any workspace of plans[i].workspace_bytes, which then
 * builds the cage adjacency itself) and the plan subdiv_refine_batch needs.
 * A fault in any mesh fails the call with that fault's status code and
 * zeroed plans. flags: 0 or SUBDIV_FLAG_REBUILD_EACH_LEVEL. */
int subdiv_plan_batch(const subdiv_mesh *meshes, const int *schemes, const int *levels, int n, uint32_t flags,
                      void *ws, size_t ws_bytes, subdiv_plan_info *plans, void *stream);

/* Refines a batch: outs[i] receives the final level of mesh i (face_verts
 * [H_L], positions [V_L*3], sized from plans[i].level[levels[i]] when
 * plans[i].levels == levels[i], else from the level sizes of a plan with
 * levels[i] levels; edge_verts and crease_sharpness are not written).
 * plans[i] is a plan of mesh i (same face_verts pointer, scheme schemes[i],
 * at least levels[i] levels, not SUBDIV_FLAG_KEEP_STATE): its cage counts
 * size every level, so the call enqueues work only (the pointer and gather
 * tables go to the device through library-owned pinned host memory, in
 * stream order). Positions may differ from the planned ones. `ws` needs
 * subdiv_batch_workspace_bound(meshes, schemes, levels, n, plans, flags)
 * bytes and is overwritten. Returns SUBDIV_STATE when a plan does not match
 * its mesh. */
int subdiv_refine_batch(const subdiv_mesh *meshes, const int *schemes, const int *levels, int n,
                        const subdiv_plan_info *plans, subdiv_level_out *outs, void *ws, size_t ws_bytes,
                        void *stream);

/* ---- optional stage timing ---------------------------------------------
 * When enabled (process-wide switch, default off), subdiv_plan and
 * subdiv_refine record a HIP event pair on their stream around every kernel
 * (or kernel group) they launch. subdiv_timing_read waits for the recorded
 * events, writes up to max_out entries aggregated by (stage, level) and
 * clears the records; it returns the number of entries written, or a
 * negative status. Stage names: "build" (cage adjacency), "rebuild" (per-level
 * generic build), "bscan" (boundary prefix), "cc_face", "cc_vertex",
 * "cc_edge" (a level refined from its own adjacency), "cc_group",
 * "cc_old_vertex", "cc_ep_vertex", "cc_edge_group" (a Catmull-Clark level
 * refined from its parent level's adjacency, one thread per parent face /
 * vertex / edge), "loop_edge", "loop_scan", "loop_vertex", "loop_face",
 * "sqrt3_count", "sqrt3_scan", "sqrt3_face", "sqrt3_vertex" (the scans give
 * the next level's edge ids), "sqrt3_trisect" (SUBDIV_SQRT3_KOBBELT's
 * trisection step), "bw_coef", "bw_face", "bw_vertex" (adjoint),
 * "batch_extract", "edge_export"; level = the level refined. */
typedef struct subdiv_stage_time {
  char name[24];
  int32_t level;
  int32_t launches;
  double total_ms;
} subdiv_stage_time;

void subdiv_timing_enable(int on);
int subdiv_timing_read(subdiv_stage_time *out, int max_out);
/* Restrict the timing to one stage name and level (level < 0: every level),
 * so that only its kernels get an event pair; NULL or "" times every stage
 * again. Process-wide, like subdiv_timing_enable. */
void subdiv_timing_select(const char *stage, int level);

/* The same records with the tuned kernel of each stage: per (stage, level,
 * kernel, element count, workgroup size), the kernel being the last tuned
 * launch inside the stage (kernel "" when the stage has none). Clears the
 * records like subdiv_timing_read; returns the entries written or a
 * negative status. */
typedef struct subdiv_kernel_time {
  char stage[24];
  char kernel[24];
  int32_t level;
  int32_t block;
  int64_t items;
  int32_t launches;
  int32_t reserved0;
  double total_ms;
} subdiv_kernel_time;
int subdiv_timing_read_kernels(subdiv_kernel_time *out, int max_out);

/* ---- launch shapes ------------------------------------------------------
 * The per-element kernels of the refinement steps and of the adjoint run
 * with a workgroup size (64, 128, 256 or 512 lanes) taken per kernel and size
 * bucket from a tuning table; the outputs do not depend on it (every lane owns
 * its element; lanes cooperate only within a wave). The table is a JSON file
 * written by the tuner (python -m paper_1809_06047_amd.tune):
 *   {"kernels": {"<kernel>": [[max_items, block], ...], ...}, ...}
 * where a launch over n elements takes the first entry with n <= max_items
 * (max_items < 0: any n; past the last entry: the last). The library reads it
 * once, at its first launch, from the path in the environment variable
 * SUBDIV_TUNING if set (empty: none), else from tuning_gfx950.json beside
 * libsubdiv.so if present; kernels without entries use 256. Process-wide. */
/* Replace the table with the file at `path` (NULL or "": no table, 256
 * everywhere). On a malformed file the table is unchanged and the call returns
 * SUBDIV_INVALID_ARG (subdiv_last_error() says why). */
int subdiv_tuning_load(const char *path);
/* Set one entry: kernel "<name>" or "*" (every kernel); max_items < 0 makes
 * `block` the kernel's only entry, else the entry with that bound is added or
 * replaced. SUBDIV_INVALID_ARG for an unknown kernel or a block other than
 * 64, 128, 256, 512. */
int subdiv_tuning_set(const char *kernel, int64_t max_items, int block);
/* The workgroup size a launch of `kernel` over `items` elements takes, or a
 * negative status for an unknown kernel. */
int subdiv_tuning_block(const char *kernel, int64_t items);
/* Where the table came from: its path, "built-in", or "set by
 * subdiv_tuning_set". Valid until the next tuning call. */
const char *subdiv_tuning_source(void);
/* Name of tunable kernel `index` (0, 1, ... until SUBDIV_INVALID_ARG) into
 * out[max_out]. */
int subdiv_tuning_kernel_name(int index, char *out, int max_out);

/* HIP error text of the last SUBDIV_HIP status on this thread, the sizes
 * behind the last SUBDIV_WORKSPACE of subdiv_refine_static, or why the last
 * subdiv_tuning_load failed ("" if none). */
const char *subdiv_last_error(void);

/* Human-readable name of a status code. */
const char *subdiv_strerror(int status);

/* Library version, 1000*major + minor (1001: seed_flags in subdiv_extraction,
 * SUBDIV_SQRT3_KOBBELT, the tuning table, subdiv_refine_static). */
int subdiv_version(void);

#ifdef __cplusplus
}
#endif
#endif /* SUBDIV_H */
