// Host runtime and C ABI of libsubdiv: size planning (closed-form counts per
// level), workspace carving, the plan (symbolic pass on the cage) and the
// per-level build/eval loop of the dynamic-topology mode (Sec. 3.6).
#include <atomic>
#include <cstring>
#include <mutex>
#include <unordered_map>
#include <string>
#include <vector>

#include "subdiv_internal.h"

using namespace subdiv;

namespace {

thread_local std::string g_last_error;

int hip_fail(hipError_t e) {
  g_last_error = hipGetErrorString(e);
  return SUBDIV_HIP;
}

#define SUBDIV_TRY(expr)                         \
  do {                                           \
    hipError_t _e = (expr);                      \
    if (_e != hipSuccess) return hip_fail(_e);   \
  } while (0)

// ---- optional stage timing (HIP events on the call's stream) ------------
struct TimingRec {
  const char *name;
  int level;
  hipEvent_t a, b;
  int key;          // tuned kernel of the stage (its last tuned launch), or -1
  long long items;  // its element count
  int block;        // and workgroup size
};
std::mutex g_tmu;
std::atomic<bool> g_timing{false};
std::vector<TimingRec> g_recs;
std::vector<hipEvent_t> g_pool;

// optional selection: only one stage (and level) is timed, so that the event
// pairs of the other stages do not sit between the kernels
std::atomic<bool> g_tsel_on{false};
char g_tsel_name[24] = "";
int g_tsel_level = -1;

hipEvent_t timing_begin(const char *name, int level, hipStream_t s) {
  if (!g_timing.load(std::memory_order_relaxed)) return nullptr;
  std::lock_guard<std::mutex> lock(g_tmu);
  if (g_tsel_on.load(std::memory_order_relaxed) &&
      (std::strcmp(name, g_tsel_name) != 0 || (g_tsel_level >= 0 && level != g_tsel_level)))
    return nullptr;
  hipEvent_t e = nullptr;
  if (!g_pool.empty()) {
    e = g_pool.back();
    g_pool.pop_back();
  } else if (hipEventCreate(&e) != hipSuccess) {
    return nullptr;
  }
  if (hipEventRecord(e, s) != hipSuccess) {
    g_pool.push_back(e);
    return nullptr;
  }
  tune_note_reset();
  return e;
}

void timing_end(hipEvent_t a, const char *name, int level, hipStream_t s) {
  if (!a) return;
  std::lock_guard<std::mutex> lock(g_tmu);
  hipEvent_t b = nullptr;
  if (!g_pool.empty()) {
    b = g_pool.back();
    g_pool.pop_back();
  } else if (hipEventCreate(&b) != hipSuccess) {
    g_pool.push_back(a);
    return;
  }
  if (hipEventRecord(b, s) != hipSuccess) {
    g_pool.push_back(a);
    g_pool.push_back(b);
    return;
  }
  TimingRec r{name, level, a, b, -1, 0, 0};
  tune_note_take(&r.key, &r.items, &r.block);
  g_recs.push_back(r);
}

#define SUBDIV_TIMED(name, level, expr)          \
  do {                                           \
    hipEvent_t _ta = timing_begin(name, level, s); \
    hipError_t _e = (expr);                      \
    if (_e != hipSuccess) return hip_fail(_e);   \
    timing_end(_ta, name, level, s);             \
  } while (0)

int status_from_faults(uint32_t f) {
  if (f & FAULT_INVALID_ARG) return SUBDIV_INVALID_ARG;
  if (f & FAULT_SCHEME_MESH) return SUBDIV_SCHEME_MESH;
  if (f & FAULT_DEGENERATE) return SUBDIV_DEGENERATE;
  if (f & FAULT_NONMANIFOLD) return SUBDIV_NONMANIFOLD;
  if (f & FAULT_BAD_CREASE) return SUBDIV_BAD_CREASE;
  return SUBDIV_OK;
}

struct Sizes {
  long long V, E, F, H, B;
  int order;
  int creases;  // level may carry creases
};

// Closed-form counts of the refined levels (index rules of Sec. 3.2, App. A, App. B).
void level_sizes(int scheme, int levels, long long V0, long long F0, long long H0, long long E0, long long B0,
                 int order0, float max_sharp, long long C0, Sizes *L) {
  const bool sqrt3 = scheme == SUBDIV_SQRT3 || scheme == SUBDIV_SQRT3_KOBBELT;
  L[0] = Sizes{V0, E0, F0, H0, B0, order0, (!sqrt3 && C0 > 0 && max_sharp > 0.f) ? 1 : 0};
  for (int k = 0; k < levels; ++k) {
    const Sizes &a = L[k];
    Sizes b{};
    if (scheme == SUBDIV_CATMULL_CLARK) {
      b = Sizes{a.V + a.F + a.E, 2 * a.E + a.H, a.H, 4 * a.H, 2 * a.B, 4, 0};
    } else if (scheme == SUBDIV_LOOP) {
      b = Sizes{a.V + a.E, 2 * a.E + 3 * a.F, 4 * a.F, 12 * a.F, 2 * a.B, 3, 0};
    } else if (scheme == SUBDIV_SQRT3_KOBBELT && k % 2 == 1) {  // trisection step: two points per boundary edge
      b = Sizes{a.V + a.F + a.B, a.E + 3 * a.F + a.B, 3 * a.F, 9 * a.F, 3 * a.B, 3, 0};
    } else {
      b = Sizes{a.V + a.F, a.E + 3 * a.F, 3 * a.F, 9 * a.F, a.B, 3, 0};
    }
    // child sharpness <= parent sharpness - 1 (Chaikin rule), so level k+1 can
    // only hold creases while the cage's largest sharpness exceeds k+1
    b.creases = (L[0].creases && (double)max_sharp > (double)(k + 1)) ? 1 : 0;
    L[k + 1] = b;
  }
}

bool sizes_fit_int32(const Sizes *L, int levels) {
  const long long lim = 0x7fffffffLL - 16;
  for (int k = 0; k <= levels; ++k) {
    const Sizes &s = L[k];
    if (s.V > lim || s.E > lim || s.F > lim || s.H > lim || 3 * s.V > lim * 2) return false;
    if (s.V + s.F + s.E > lim) return false;
  }
  return true;
}

// ---- workspace layout --------------------------------------------------
struct Carver {
  size_t at = 0;
  size_t take(size_t bytes) {
    at = (at + 255) & ~size_t(255);
    const size_t p = at;
    at += bytes;
    return p;
  }
};

struct AdjOffsets {
  size_t fv, twin, eid, vhe, e2h, bscan, sig, vcr;
};

struct Layout {
  size_t info, info2;
  // level-0 region (depends on V0, F0, H0, C0 only)
  size_t nval, rowptr, cursor, inc, cand, cntlo, ebase, bflag, sigcnt, partials0;
  size_t hface0;
  AdjOffsets adj0;
  size_t sel_x[2], sel_q, sel_vnew, sel_fnew, sel_onew, sel_flag, sel_cnew, sel_totals, sel_x0;  // selective extraction
  size_t sel_qadd, sel_changed;
  size_t level0_end;
  // per-level regions
  AdjOffsets slot[3];  // adjacency of levels k-2, k-1, k rotate through these (index level % 3)
  size_t hs, term0;    // half rings / corner-0 terms of the corner-class kernels
  size_t tbase;        // edge bases of the next level (triangle schemes with carried adjacency)
  size_t tbase2;       // Loop, second step from below: the edge bases of level L-2 beside level L-3's
  size_t tslot, trank, tnb;  // sqrt(3) trisection steps: boundary slot and rank per face, boundary neighbours
  size_t tbase3, tmask;      // and, for the carried adjacency, run bases and per-face point kinds
  size_t partials;     // scan partials of every level after the cage
  size_t bnval, browptr, bcursor, binc, bcand, bcntlo, bebase, bbflag, bsigcnt;  // rebuild scratch
  size_t mfv[2], mP[2];
  // SUBDIV_FLAG_KEEP_STATE: adjacency of every level 1..L-1 and the backward scratch
  AdjOffsets keep[SUBDIV_MAX_LEVELS + 1];
  size_t bg[2], bterm;
  size_t kcoef[SUBDIV_MAX_LEVELS + 1];  // kept state: the adjoint's vertex-rule coefficients of level k
  size_t total;
};

AdjOffsets carve_adj(Carver &c, long long V, long long E, long long H, bool creases, bool with_fv) {
  AdjOffsets a{};
  a.fv = with_fv ? c.take(4 * H) : 0;
  a.twin = c.take(4 * H);
  a.eid = c.take(4 * H);
  a.vhe = c.take(4 * V);
  a.e2h = c.take(4 * (E > 0 ? E : 1));
  a.bscan = c.take(4 * (E + 1));
  a.sig = creases ? c.take(8 * (E > 0 ? E : 1)) : 0;
  a.vcr = creases ? c.take(16 * V) : 0;
  return a;
}

// Levels >= 1 are built from scratch by the generic mapped product when the
// caller asks for it; otherwise every scheme carries each level's adjacency
// over in closed form from the level it was refined from.
bool rebuilds_levels(int scheme, uint32_t flags) {
  (void)scheme;
  return (flags & SUBDIV_FLAG_REBUILD_EACH_LEVEL) != 0;
}

// The last two Loop or sqrt(3) steps both run from two levels below them:
// L >= 4 (so the step before the last reads a refined level, L-3 >= 1) and
// no creases on levels L-2 and L-1
// The last Loop or sqrt(3) step from level L-2 (level L-1's adjacency never
// built): not when every level's state is kept
// (sqrt(3) with the boundary cycle steps level by level)
bool tri_lag(int scheme, uint32_t flags, int levels, const Sizes *L) {
  return (scheme == SUBDIV_LOOP || scheme == SUBDIV_SQRT3) && !rebuilds_levels(scheme, flags) &&
         !(flags & SUBDIV_FLAG_KEEP_STATE) && levels >= 3 && !L[levels - 1].creases;
}
// and the step before it from level L-3 too
bool tri_lag2(int scheme, uint32_t flags, int levels, const Sizes *L) {
  return tri_lag(scheme, flags, levels, L) && levels >= 4 && !L[levels - 2].creases;
}

Layout make_layout(int scheme, int levels, uint32_t flags, const Sizes *L, long long C0) {
  Layout y{};
  Carver c;
  const long long V0 = L[0].V, H0 = L[0].H;
  y.info = c.take(sizeof(DeviceInfo));
  y.info2 = c.take(sizeof(DeviceInfo));
  y.nval = c.take(4 * (V0 + 1));
  y.rowptr = c.take(4 * (V0 + 1));
  y.cursor = c.take(4 * V0);
  y.inc = c.take(4 * H0);
  y.cand = c.take(8 * H0);
  y.cntlo = c.take(4 * (V0 + 1));
  y.ebase = c.take(4 * (V0 + 1));
  y.bflag = c.take(4 * (H0 + 1));
  y.sigcnt = c.take(4 * H0);
  y.partials0 = c.take(4 * (scan_partials_ints(V0 > H0 ? V0 : H0) + 8));
  y.hface0 = c.take(4 * H0);
  // level-0 adjacency: edge-indexed arrays sized by H0 >= E0
  y.adj0 = carve_adj(c, V0, H0, H0, C0 > 0, false);
  const long long F0 = L[0].F;
  y.sel_x[0] = c.take(4 * V0);
  y.sel_x[1] = c.take(4 * V0);
  y.sel_q = c.take(4 * F0);
  y.sel_vnew = c.take(4 * (V0 + 1));
  y.sel_fnew = c.take(4 * (F0 + 1));
  y.sel_onew = c.take(4 * (F0 + 1));
  y.sel_flag = c.take(4 * ((F0 > H0 ? F0 : H0) + 1));
  y.sel_cnew = c.take(4 * (H0 + 1));
  y.sel_totals = c.take(16);
  y.sel_x0 = c.take(V0);
  y.sel_qadd = c.take(4 * F0);
  y.sel_changed = c.take(4 * kPinchPasses);
  y.level0_end = c.at;
  // everything below may depend on the level count and on E0
  long long maxn = 1;
  for (int k = 1; k <= levels; ++k) {
    maxn = L[k].V > maxn ? L[k].V : maxn;
    maxn = L[k].E > maxn ? L[k].E : maxn;
    // a trisection step scans two counts per face
    if (scheme == SUBDIV_SQRT3_KOBBELT && k % 2 == 1 && k < levels) maxn = 2 * L[k].F > maxn ? 2 * L[k].F : maxn;
  }
  y.partials = c.take(4 * (scan_partials_ints(maxn) + 8));
  if (levels >= 2) {
    const bool rebuild = rebuilds_levels(scheme, flags);
    // the last Loop or sqrt(3) step from level levels-2: level levels-1's
    // adjacency and face table are never held in the workspace (only its
    // positions)
    const bool keep = (flags & SUBDIV_FLAG_KEEP_STATE) != 0;
    const bool loop_lag = tri_lag(scheme, flags, levels, L);
    const int top = loop_lag ? levels - 1 : levels;  // levels 1 .. top-1 have adjacency slots and face tables
    long long mV = 0, mE = 0, mH = 0, mF = 0, mVp = 0;
    bool cr = false;
    for (int k = 1; k < top; ++k) {
      mV = L[k].V > mV ? L[k].V : mV;
      mE = L[k].E > mE ? L[k].E : mE;
      mH = L[k].H > mH ? L[k].H : mH;
      mF = L[k].F > mF ? L[k].F : mF;
      cr = cr || L[k].creases;
    }
    for (int k = 1; k < levels; ++k) mVp = L[k].V > mVp ? L[k].V : mVp;
    const bool cc_carry = scheme == SUBDIV_CATMULL_CLARK && !rebuild;
    // rotating adjacency slots; with the state kept every level has its own region instead
    const int nslots = keep ? 0 : (cc_carry ? 3 : 2);
    for (int s = 0; s < nslots; ++s) y.slot[s] = carve_adj(c, mV, mE, mH, cr, true);
    if (cc_carry && levels >= 4) {
      y.hs = c.take(24 * mE);
      y.term0 = c.take(12 * mF);
    }

    if (rebuild) {
      y.bnval = c.take(4 * (mV + 1));
      y.browptr = c.take(4 * (mV + 1));
      y.bcursor = c.take(4 * mV);
      y.binc = c.take(4 * mH);
      y.bcand = c.take(8 * mH);
      y.bcntlo = c.take(4 * (mV + 1));
      y.bebase = c.take(4 * (mV + 1));
      y.bbflag = c.take(4 * (mH + 1));
      y.bsigcnt = c.take(4 * mH);
    }
    for (int s = 0; s < 2; ++s) {
      if (!keep) y.mfv[s] = c.take(4 * (mH > 0 ? mH : 1));  // (kept levels hold their own face tables)
      y.mP[s] = c.take(12 * mVp);
    }
  }
  if (scheme != SUBDIV_CATMULL_CLARK && levels >= 1) {
    // edge bases of the triangle levels (Loop: one entry per edge, sqrt(3):
    // per face) of every level that is refined further, and with Loop
    // creases on the last level refined, of that level too (its bases give
    // the ids of the inherited sharpness)
    long long mX = 0;
    const int last = (scheme == SUBDIV_LOOP && L[levels - 1].creases) ? levels : levels - 1;
    for (int k = 0; k < last; ++k) {
      const long long x = scheme == SUBDIV_LOOP ? L[k].E : L[k].F;
      mX = x > mX ? x : mX;
    }
    y.tbase = c.take(4 * (mX + 1));
    if (tri_lag2(scheme, flags, levels, L))
      y.tbase2 = c.take(4 * ((scheme == SUBDIV_LOOP ? L[levels - 2].E : L[levels - 2].F) + 1));
  }
  if (scheme == SUBDIV_SQRT3_KOBBELT && levels >= 2) {  // trisection steps from the odd levels
    long long tV = 1, tF = 1;
    for (int k = 1; k < levels; k += 2) {
      tV = L[k].V > tV ? L[k].V : tV;
      tF = L[k].F > tF ? L[k].F : tF;
    }
    y.tslot = c.take(4 * tF);
    y.trank = c.take(4 * (tF + 1));
    y.tnb = c.take(8 * tV);
    y.tbase3 = c.take(4 * (2 * tF + 1));  // carried adjacency: edge counts of the p / face-point and q runs
    y.tmask = c.take(tF);
  }
  if (flags & SUBDIV_FLAG_KEEP_STATE) {
    long long gV = L[0].V, gH = L[0].H;
    for (int k = 1; k < levels; ++k) {
      y.keep[k] = carve_adj(c, L[k].V, L[k].E, L[k].H, L[k].creases != 0, true);
      gH = L[k].H > gH ? L[k].H : gH;
    }
    for (int k = 1; k <= levels; ++k) gV = L[k].V > gV ? L[k].V : gV;
    y.bg[0] = c.take(12 * gV);
    y.bg[1] = c.take(12 * gV);
    y.bterm = c.take(12 * gH);
    if (scheme == SUBDIV_CATMULL_CLARK)  // the adjoint covers Catmull-Clark
      for (int k = 0; k < levels; ++k) y.kcoef[k] = c.take(16 * L[k].V);
  }
  y.total = c.at + 256;
  return y;
}

// What the library knows about each workspace it has been handed (host-side
// records; the device memory itself is the caller's):
//   plan  - stamp of the plan whose cage adjacency the level-0 region holds
//           (written by subdiv_plan or by a refinement that rebuilt it);
//   kept  - stamp of the SUBDIV_FLAG_KEEP_STATE plan whose every-level state
//           a completed subdiv_refine enqueued into it (0: none);
//   coef  - stamp of the plan whose adjoint vertex-rule coefficients it holds.
// The coefficients depend on the topology and the creases only, so they are
// fixed by the plan: the first backward pass with a plan's workspace writes
// them into the kept state, and every later one with the same plan reads
// them. Callers that keep the state only for positions-only or vertex-data
// evaluation never pay for them. subdiv_state_destroy drops a record.
struct WsRecord {
  uint64_t plan = 0, kept = 0, coef = 0;
};
std::mutex g_ws_mu;
std::unordered_map<const void *, WsRecord> g_ws;

// one counter for every plan and batch plan, so that no two share a stamp
uint64_t next_stamp() {
  static std::atomic<uint64_t> stamp{1};
  return stamp++;
}

WsRecord ws_record(const void *ws) {
  std::lock_guard<std::mutex> lock(g_ws_mu);
  const auto it = g_ws.find(ws);
  return it == g_ws.end() ? WsRecord{} : it->second;
}

// a plan (re)wrote the level-0 region: nothing else it held is valid any more
void ws_planned(const void *ws, uint64_t stamp) {
  std::lock_guard<std::mutex> lock(g_ws_mu);
  g_ws[ws] = WsRecord{stamp, 0, 0};
}

// a refinement wrote the level-0 region (reused or rebuilt) and, with the
// state kept, every level's topology
void ws_refined(const void *ws, uint64_t stamp, bool keep) {
  std::lock_guard<std::mutex> lock(g_ws_mu);
  g_ws[ws] = WsRecord{stamp, keep ? stamp : 0, 0};
}

void ws_coefs(const void *ws, uint64_t stamp) {
  std::lock_guard<std::mutex> lock(g_ws_mu);
  g_ws[ws].coef = stamp;
}

// a batch overwrote [ws, ws + bytes): every record inside is stale
void ws_forget_range(const void *ws, size_t bytes) {
  std::lock_guard<std::mutex> lock(g_ws_mu);
  const char *lo = static_cast<const char *>(ws), *hi = lo + bytes;
  for (auto it = g_ws.begin(); it != g_ws.end();) {
    const char *p = static_cast<const char *>(it->first);
    if (p >= lo && p < hi)
      it = g_ws.erase(it);
    else
      ++it;
  }
}

bool state_kept(const subdiv_plan_info *plan, const void *ws) {
  return plan->priv_stamp != 0 && ws_record(ws).kept == plan->priv_stamp;
}

template <class T>
T *at(void *ws, size_t off) {
  return reinterpret_cast<T *>(static_cast<char *>(ws) + off);
}

Adj adj_at(void *ws, const AdjOffsets &o, long long E, bool creases) {
  Adj a{};
  a.fv = o.fv ? at<int32_t>(ws, o.fv) : nullptr;
  a.twin = at<int32_t>(ws, o.twin);
  a.eid = at<int32_t>(ws, o.eid);
  a.vhe = at<int32_t>(ws, o.vhe);
  a.e2h = at<int32_t>(ws, o.e2h);
  a.bscan = at<int32_t>(ws, o.bscan);
  a.sig = creases && o.sig ? at<double>(ws, o.sig) : nullptr;
  a.vcr = creases && o.vcr ? at<int4>(ws, o.vcr) : nullptr;
  a.E = (int32_t)E;
  return a;
}

BuildScratch scratch0(void *ws, const Layout &y) {
  BuildScratch b{};
  b.nval = at<int32_t>(ws, y.nval);
  b.rowptr = at<int32_t>(ws, y.rowptr);
  b.cursor = at<int32_t>(ws, y.cursor);
  b.inc = at<int32_t>(ws, y.inc);
  b.cand = at<int32_t>(ws, y.cand);
  b.cntlo = at<int32_t>(ws, y.cntlo);
  b.ebase = at<int32_t>(ws, y.ebase);
  b.bflag = at<int32_t>(ws, y.bflag);
  b.sigcnt = at<int32_t>(ws, y.sigcnt);
  b.partials = at<int32_t>(ws, y.partials0);
  return b;
}

SelectScratch select_scratch(void *ws, const Layout &y) {
  SelectScratch w{};
  w.x[0] = at<int32_t>(ws, y.sel_x[0]);
  w.x[1] = at<int32_t>(ws, y.sel_x[1]);
  w.q = at<int32_t>(ws, y.sel_q);
  w.vnew = at<int32_t>(ws, y.sel_vnew);
  w.fnew = at<int32_t>(ws, y.sel_fnew);
  w.onew = at<int32_t>(ws, y.sel_onew);
  w.flag = at<int32_t>(ws, y.sel_flag);
  w.cnew = at<int32_t>(ws, y.sel_cnew);
  w.partials = at<int32_t>(ws, y.partials0);
  w.totals = at<int32_t>(ws, y.sel_totals);
  w.seed0 = at<uint8_t>(ws, y.sel_x0);
  w.qadd = at<int32_t>(ws, y.sel_qadd);
  w.changed = at<int32_t>(ws, y.sel_changed);
  return w;
}

BuildScratch scratch_rebuild(void *ws, const Layout &y) {
  BuildScratch b{};
  b.nval = at<int32_t>(ws, y.bnval);
  b.rowptr = at<int32_t>(ws, y.browptr);
  b.cursor = at<int32_t>(ws, y.bcursor);
  b.inc = at<int32_t>(ws, y.binc);
  b.cand = at<int32_t>(ws, y.bcand);
  b.cntlo = at<int32_t>(ws, y.bcntlo);
  b.ebase = at<int32_t>(ws, y.bebase);
  b.bflag = at<int32_t>(ws, y.bbflag);
  b.sigcnt = at<int32_t>(ws, y.bsigcnt);
  b.partials = at<int32_t>(ws, y.partials);
  return b;
}

Topo cage_topo(const subdiv_mesh *m, long long H, void *ws, const Layout &y) {
  Topo t{};
  t.V = m->num_vertices;
  t.F = m->num_faces;
  t.H = (int32_t)H;
  t.order = m->face_offsets ? 0 : m->face_order;
  t.off = m->face_offsets;
  t.hface = m->face_offsets ? at<int32_t>(ws, y.hface0) : nullptr;
  t.fv = m->face_verts;
  return t;
}

int check_mesh_args(const subdiv_mesh *m, int scheme, int levels) {
  if (!m || !m->face_verts || !m->positions) return SUBDIV_INVALID_ARG;
  if (reinterpret_cast<uintptr_t>(m->face_verts) % 16 != 0) return SUBDIV_INVALID_ARG;  // read as int4 rows
  if (scheme < 0 || scheme > SUBDIV_SQRT3_KOBBELT || levels < 1 || levels > SUBDIV_MAX_LEVELS) return SUBDIV_INVALID_ARG;
  if (m->num_vertices < 1 || m->num_faces < 1) return SUBDIV_INVALID_ARG;
  if (!m->face_offsets && m->face_order != 3 && m->face_order != 4) return SUBDIV_INVALID_ARG;
  if (m->face_offsets && m->num_halfedges < 3) return SUBDIV_INVALID_ARG;
  if (m->num_creases < 0 || (m->num_creases > 0 && (!m->crease_verts || !m->crease_sharpness)))
    return SUBDIV_INVALID_ARG;
  if (m->num_creases > 0 && (scheme == SUBDIV_SQRT3 || scheme == SUBDIV_SQRT3_KOBBELT))
    return SUBDIV_INVALID_ARG;  // creases: CC and Loop
  return SUBDIV_OK;
}

long long cage_H(const subdiv_mesh *m) {
  return m->face_offsets ? (long long)m->num_halfedges : (long long)m->num_faces * m->face_order;
}

// Level-0 build: validation pass (phase A) then the adjacency (phase B).
hipError_t build_level0_faces(const subdiv_mesh *m, int scheme, const Topo &t, void *ws, const Layout &y,
                              hipStream_t s) {
  DeviceInfo *info = at<DeviceInfo>(ws, y.info);
  hipError_t err;
  BuildScratch b = scratch0(ws, y);
  Adj a = adj_at(ws, y.adj0, t.H, m->num_creases > 0);
  // one launch clears the fault word and counters, the valence counts and
  // incidence cursors, and the edge-indexed crease state (E <= H)
  ZeroRegions z{};
  z.p[0] = reinterpret_cast<int32_t *>(info);
  z.n[0] = sizeof(DeviceInfo) / 4;
  z.p[1] = b.nval;
  z.n[1] = t.V + 1ll;
  z.p[2] = b.cursor;
  z.n[2] = t.V;
  z.count = 3;
  if (a.sig) {
    z.p[3] = reinterpret_cast<int32_t *>(a.sig);
    z.n[3] = 2ll * t.H;
    z.p[4] = b.sigcnt;
    z.n[4] = t.H;
    z.count = 5;
  }
  if ((err = launch_zero_regions(z, s)) != hipSuccess) return err;
  return build_faces(t, scheme, b, info, s, true);
}

// Catmull-Clark with the adjacency carried over in closed form: step 0 on
// the cage adjacency, steps k >= 1 from the parent level's adjacency. Level
// k's own adjacency is written during step k when a later step or the
// adjoint reads it. With SUBDIV_FLAG_KEEP_STATE every level keeps its face
// table, adjacency and sharpness in its own region (y.keep[k]); otherwise
// three slots rotate. positions_only re-evaluates the positions of a
// refinement whose state is kept (static topology): only positions are
// written, every other array is read from the kept state.
int refine_cc_carried(const subdiv_mesh *mesh, const subdiv_level_out *outs, void *ws, const Layout &y,
                      const Sizes *L, int levels, uint32_t flags, Topo t, Adj a, const float *P, bool positions_only,
                      hipStream_t s) {
  (void)mesh;
  const bool keep = (flags & SUBDIV_FLAG_KEEP_STATE) != 0;
  auto level_adj = [&](int k, bool creases) -> Adj {
    return adj_at(ws, keep ? y.keep[k] : y.slot[k % 3], L[k].E, creases);
  };
  const bool emit = !positions_only;
  const bool final0 = (levels == 1);
  CCStep c{};
  c.t = t;
  c.a = a;
  c.P = P;
  c.fv1 = (final0 && emit) ? outs[1].face_verts : nullptr;
  c.P1 = outs[1].positions ? outs[1].positions : at<float>(ws, y.mP[1]);
  c.has_bnd = L[0].B > 0;
  c.creases = L[0].creases && a.sig != nullptr;
  c.creases1 = c.creases && L[1].creases;
  if (c.creases1 && emit) c.sig1 = final0 ? outs[1].crease_sharpness : level_adj(1, true).sig;
  if (outs[1].edge_verts && emit) SUBDIV_TIMED("edge_export", 0, launch_edge_export(t, a, outs[1].edge_verts, s));
  SUBDIV_TIMED("cc_face", 0, cc_launch(CC_FACE, c, s));
  SUBDIV_TIMED("cc_vertex", 0, cc_launch(CC_VERTEX, c, s));
  SUBDIV_TIMED("cc_edge", 0, cc_launch(CC_EDGE, c, s));
  if (!final0 && c.sig1 && outs[1].crease_sharpness)
    SUBDIV_TRY(hipMemcpyAsync(outs[1].crease_sharpness, c.sig1, 8 * L[1].E, hipMemcpyDeviceToDevice, s));
  Topo tm = t;
  Adj am = a;
  Adj ag{};  // grandparent adjacency (levels >= 1 only)
  const double *sig_cur = (c.creases1 && !final0) ? level_adj(1, true).sig : nullptr;
  P = c.P1;
  for (int k = 1; k < levels; ++k) {
    const bool final = (k == levels - 1);
    const Adj slotk = level_adj(k, L[k].creases);
    LagStep g{};
    g.tm = tm;
    g.am = am;
    g.bnd = L[0].B > 0;
    g.Vk = (int32_t)L[k].V;
    g.Fk = (int32_t)L[k].F;
    g.Ek = (int32_t)L[k].E;
    g.Pk = P;
    g.sigk = L[k].creases ? sig_cur : nullptr;
    g.vcrk = (g.sigk && emit) ? slotk.vcr : nullptr;
    g.P1 = outs[k + 1].positions ? outs[k + 1].positions : at<float>(ws, y.mP[(k + 1) & 1]);
    g.fv1 = (final && emit) ? outs[levels].face_verts : nullptr;
    if (emit) g.fvk = keep ? slotk.fv : (outs[k].face_verts ? outs[k].face_verts : (final ? nullptr : slotk.fv));
    if (emit && (!final || keep)) {  // level k's adjacency: read by step k+1 or by the adjoint
      g.ak = slotk;
      g.ak.fv = nullptr;
      g.ak.sig = nullptr;
      g.ak.vcr = nullptr;
      if (!g.bnd) g.ak.bscan = nullptr;
    }
    if (emit && g.sigk && L[k + 1].creases)
      g.sig1 = final ? outs[levels].crease_sharpness : level_adj(k + 1, true).sig;
    g.edges_k = emit ? outs[k + 1].edge_verts : nullptr;
    if (k >= 3) {
      // quad parent and grandparent: rings from corner classes
      Lag2Step g2{};
      g2.s = g;
      g2.Vg = (int32_t)L[k - 2].V;
      g2.Fg = (int32_t)L[k - 2].F;
      g2.Eg = (int32_t)L[k - 2].E;
      g2.VFg = g2.Vg + g2.Fg;
      if (k >= 4) {  // level g = k-2 was itself refined from quads
        g2.Vq = (int32_t)L[k - 3].V;
        g2.Fq = (int32_t)L[k - 3].F;
      }
      g2.vhe_g = ag.vhe;
      g2.twin_g = ag.twin;
      g2.e2h_g = ag.e2h;
      g2.bscan_g = g.bnd ? ag.bscan : nullptr;
      g2.hs = at<float>(ws, y.hs);
      g2.term0 = at<float>(ws, y.term0);
      SUBDIV_TIMED("cc_group", k, lag2_launch(LAG2_GROUP, g2, s));
      SUBDIV_TIMED("cc_ep_vertex", k, lag2_launch(LAG2_COMBINE, g2, s));
      SUBDIV_TIMED("cc_old_vertex", k, lag2_launch(LAG2_OLDER, g2, s));
    } else {
      SUBDIV_TIMED("cc_group", k, lag_launch(LAG_GROUP, g, s));
      SUBDIV_TIMED("cc_old_vertex", k, lag_launch(LAG_VERTEX, g, s));
    }
    SUBDIV_TIMED("cc_edge_group", k, lag_launch(LAG_EDGE, g, s));
    if (emit && keep && outs[k].face_verts)
      SUBDIV_TRY(hipMemcpyAsync(outs[k].face_verts, slotk.fv, 4 * L[k].H, hipMemcpyDeviceToDevice, s));
    if (!final && g.sig1 && outs[k + 1].crease_sharpness)
      SUBDIV_TRY(hipMemcpyAsync(outs[k + 1].crease_sharpness, g.sig1, 8 * L[k + 1].E, hipMemcpyDeviceToDevice, s));
    tm = Topo{(int32_t)L[k].V, (int32_t)L[k].F, (int32_t)L[k].H, 4, nullptr, nullptr, emit ? g.fvk : slotk.fv};
    ag = am;
    am = slotk;
    sig_cur = emit ? g.sig1 : ((!final && L[k + 1].creases) ? level_adj(k + 1, true).sig : nullptr);
    P = g.P1;
  }
  return SUBDIV_OK;
}

// Loop and sqrt(3) positions from the kept state (static topology, Sec. 3.6):
// every level's face table and adjacency (and Loop's sharpness) are in the
// levels' own regions, so each step runs the point kernels of the per-level
// path with every topology output switched off: the same kernels on the same
// operands as the refinement that kept the state, so the same bits.
int refine_tri_kept(int scheme, const subdiv_level_out *outs, void *ws, const Layout &y, const Sizes *L, int levels,
                    Topo t, Adj a, const float *P, hipStream_t s) {
  Adj aprev{};
  for (int k = 0; k < levels; ++k) {
    const bool final = (k == levels - 1);
    float *P1 = outs[k + 1].positions ? outs[k + 1].positions : at<float>(ws, y.mP[(k + 1) & 1]);
    if (final) P1 = outs[k + 1].positions;
    TriStep c{t, a, P, nullptr, P1, Adj{}, nullptr, (int32_t)L[k].B, k >= 1 ? (int32_t)L[k - 1].V : 0, aprev,
              k >= 2 ? (int32_t)L[k - 2].V : 0};
    if (scheme == SUBDIV_LOOP) {
      SUBDIV_TIMED("loop_edge", k, tri_launch(LOOP_EDGE, c, s));
      SUBDIV_TIMED("loop_vertex", k, tri_launch(LOOP_VERTEX, c, s));
      if (L[k].creases && a.sig && a.vcr) SUBDIV_TIMED("loop_crease", k, loop_crease_launch(c, nullptr, s));
    } else {
      SUBDIV_TIMED("sqrt3_vertex", k, tri_launch(SQRT3_VERTEX, c, s));
      SUBDIV_TIMED("sqrt3_face", k, tri_launch(SQRT3_FACE, c, s));
    }
    if (!final) {
      aprev = a;
      a = adj_at(ws, y.keep[k + 1], L[k + 1].E, L[k + 1].creases != 0);
      t = Topo{(int32_t)L[k + 1].V, (int32_t)L[k + 1].F, (int32_t)L[k + 1].H, 3, nullptr, nullptr,
               at<int32_t>(ws, y.keep[k + 1].fv)};
    }
    P = P1;
  }
  return SUBDIV_OK;
}

// The symbolic pass on a cage, enqueued only: validation of faces and
// indices and the valence; then the adjacency, edge ids and creases, whose
// kernels do nothing once a fault is recorded; for Loop and sqrt(3) refined
// twice or more, the count of two-face components. Counts and faults are
// left in the level-0 region's DeviceInfo for one read-back.
int plan_enqueue(const subdiv_mesh *mesh, int scheme, int levels, void *ws, const Layout &y0, hipStream_t s) {
  const long long H0 = cage_H(mesh);
  const Topo t = cage_topo(mesh, H0, ws, y0);
  DeviceInfo *dinfo = at<DeviceInfo>(ws, y0.info);
  SUBDIV_TIMED("build", 0, build_level0_faces(mesh, scheme, t, ws, y0, s));
  BuildScratch b = scratch0(ws, y0);
  Adj a0 = adj_at(ws, y0.adj0, H0, mesh->num_creases > 0);
  SUBDIV_TIMED("build", 0, build_adjacency(t, scheme, b, a0, dinfo, s));
  SUBDIV_TIMED("build", 0,
               build_creases(t, b, a0, mesh->num_creases, mesh->crease_verts, mesh->crease_sharpness, dinfo, s));
  if (scheme != SUBDIV_CATMULL_CLARK && levels >= 2) SUBDIV_TIMED("build", 0, count_pillows(t, a0, dinfo, s));
  return SUBDIV_OK;
}

int plan_status(const DeviceInfo &h, int scheme, int levels) {
  const int st = status_from_faults(h.faults);
  if (st != SUBDIV_OK) return st;
  // a two-face component refined by Loop or sqrt(3) is not manifold after one level
  if (scheme != SUBDIV_CATMULL_CLARK && levels >= 2 && h.num_pillows > 0) return SUBDIV_NONMANIFOLD;
  return SUBDIV_OK;
}

// A plan from the cage's counts: the closed-form sizes of every level, the
// workspace refine needs, and a fresh stamp. `ws` is the workspace whose
// level-0 region holds the cage's adjacency, or nullptr.
int fill_plan(subdiv_plan_info *plan, const subdiv_mesh *mesh, int scheme, int levels, uint32_t flags, long long E0,
              long long B0, float max_sharp, int max_valence, const void *ws) {
  std::memset(plan, 0, sizeof(*plan));
  const long long H0 = cage_H(mesh);
  Sizes L[SUBDIV_MAX_LEVELS + 1];
  level_sizes(scheme, levels, mesh->num_vertices, mesh->num_faces, H0, E0, B0, mesh->face_offsets ? 0 : mesh->face_order,
              max_sharp, mesh->num_creases, L);
  if (!sizes_fit_int32(L, levels)) return SUBDIV_INVALID_ARG;
  const Layout y = make_layout(scheme, levels, flags, L, mesh->num_creases);
  plan->scheme = scheme;
  plan->levels = levels;
  plan->flags = flags;
  plan->max_valence = max_valence;
  plan->max_sharpness = max_sharp;
  for (int k = 0; k <= levels; ++k) {
    subdiv_level_info &li = plan->level[k];
    li.num_vertices = L[k].V;
    li.num_edges = L[k].E;
    li.num_faces = L[k].F;
    li.num_halfedges = L[k].H;
    li.num_boundary_edges = L[k].B;
    li.face_order = L[k].order;
    long long cmax = 0;
    if (L[k].creases) {
      cmax = (long long)mesh->num_creases << (k < 30 ? k : 30);
      if (cmax > L[k].E) cmax = L[k].E;
    }
    li.max_creases = (int32_t)cmax;
  }
  plan->workspace_bytes = y.total;
  plan->priv_mesh_verts = mesh->face_verts;
  plan->priv_ws = ws;
  plan->priv_stamp = next_stamp();
  return SUBDIV_OK;
}

int refine_impl(const subdiv_mesh *mesh, const subdiv_plan_info *plan, subdiv_level_out *outs, void *ws,
                size_t ws_bytes, void *stream);

}  // namespace

namespace subdiv {
void subdiv_set_error(const char *msg) { g_last_error = msg ? msg : ""; }
}  // namespace subdiv

// ---- the C ABI ---------------------------------------------------------
extern "C" {

int subdiv_version(void) { return 1001; }

void subdiv_timing_enable(int on) { g_timing.store(on != 0); }

void subdiv_timing_select(const char *stage, int level) {
  std::lock_guard<std::mutex> lock(g_tmu);
  if (!stage || !*stage) {
    g_tsel_on.store(false);
    g_tsel_name[0] = 0;
    g_tsel_level = -1;
    return;
  }
  std::strncpy(g_tsel_name, stage, sizeof(g_tsel_name) - 1);
  g_tsel_name[sizeof(g_tsel_name) - 1] = 0;
  g_tsel_level = level;
  g_tsel_on.store(true);
}

int subdiv_timing_read(subdiv_stage_time *out, int max_out) {
  if (!out || max_out < 0) return SUBDIV_INVALID_ARG;
  std::lock_guard<std::mutex> lock(g_tmu);
  int n = 0;
  hipError_t first = hipSuccess;
  for (const TimingRec &r : g_recs) {
    float ms = 0.f;
    hipError_t e = hipEventSynchronize(r.b);
    if (e == hipSuccess) e = hipEventElapsedTime(&ms, r.a, r.b);
    if (e != hipSuccess && first == hipSuccess) first = e;
    int i = 0;
    for (; i < n; ++i)
      if (out[i].level == r.level && std::strncmp(out[i].name, r.name, sizeof(out[i].name)) == 0) break;
    if (i == n) {
      if (n == max_out) continue;
      std::memset(&out[n], 0, sizeof(out[n]));
      std::strncpy(out[n].name, r.name, sizeof(out[n].name) - 1);
      out[n].level = r.level;
      ++n;
    }
    out[i].launches += 1;
    out[i].total_ms += ms;
    g_pool.push_back(r.a);
    g_pool.push_back(r.b);
  }
  g_recs.clear();
  if (first != hipSuccess) return hip_fail(first);
  return n;
}

int subdiv_timing_read_kernels(subdiv_kernel_time *out, int max_out) {
  if (!out || max_out < 0) return SUBDIV_INVALID_ARG;
  std::lock_guard<std::mutex> lock(g_tmu);
  int n = 0;
  hipError_t first = hipSuccess;
  for (const TimingRec &r : g_recs) {
    float ms = 0.f;
    hipError_t e = hipEventSynchronize(r.b);
    if (e == hipSuccess) e = hipEventElapsedTime(&ms, r.a, r.b);
    if (e != hipSuccess && first == hipSuccess) first = e;
    const char *kname = r.key >= 0 ? tune_key_name(r.key) : "";
    int i = 0;
    for (; i < n; ++i)
      if (out[i].level == r.level && out[i].items == r.items && out[i].block == r.block &&
          std::strncmp(out[i].stage, r.name, sizeof(out[i].stage)) == 0 &&
          std::strncmp(out[i].kernel, kname, sizeof(out[i].kernel)) == 0)
        break;
    if (i == n) {
      if (n == max_out) continue;
      std::memset(&out[n], 0, sizeof(out[n]));
      std::strncpy(out[n].stage, r.name, sizeof(out[n].stage) - 1);
      std::strncpy(out[n].kernel, kname, sizeof(out[n].kernel) - 1);
      out[n].level = r.level;
      out[n].items = r.items;
      out[n].block = r.block;
      ++n;
    }
    out[i].launches += 1;
    out[i].total_ms += ms;
    g_pool.push_back(r.a);
    g_pool.push_back(r.b);
  }
  g_recs.clear();
  if (first != hipSuccess) return hip_fail(first);
  return n;
}

const char *subdiv_last_error(void) { return g_last_error.c_str(); }

const char *subdiv_strerror(int st) {
  switch (st) {
    case SUBDIV_OK: return "ok";
    case SUBDIV_INVALID_ARG: return "invalid argument";
    case SUBDIV_SCHEME_MESH: return "scheme needs a triangle mesh";
    case SUBDIV_NONMANIFOLD: return "non-manifold or inconsistently oriented mesh";
    case SUBDIV_DEGENERATE: return "degenerate face or isolated vertex";
    case SUBDIV_BAD_CREASE: return "bad crease";
    case SUBDIV_WORKSPACE: return "workspace too small";
    case SUBDIV_HIP: return "HIP runtime error";
    case SUBDIV_STATE: return "plan does not match the call";
    default: return "unknown status";
  }
}

size_t subdiv_workspace_bound(int32_t V, int32_t F, int64_t H, int32_t C, int scheme, int levels, uint32_t flags) {
  if (V < 1 || F < 1 || H < 3 || levels < 1 || levels > SUBDIV_MAX_LEVELS || scheme < 0 ||
      scheme > SUBDIV_SQRT3_KOBBELT)
    return 0;
  Sizes L[SUBDIV_MAX_LEVELS + 1];
  // E0 <= H0 and B0 <= H0 bound every later level from above
  level_sizes(scheme, levels, V, F, H, H, H, 0, C > 0 ? 1e30f : 0.f, C, L);
  if (!sizes_fit_int32(L, levels)) return 0;
  return make_layout(scheme, levels, flags, L, C).total;
}

int subdiv_plan(const subdiv_mesh *mesh, int scheme, int levels, uint32_t flags, void *ws, size_t ws_bytes,
                subdiv_plan_info *plan, void *stream) {
  if (!plan) return SUBDIV_INVALID_ARG;
  std::memset(plan, 0, sizeof(*plan));
  int st = check_mesh_args(mesh, scheme, levels);
  if (st != SUBDIV_OK) return st;
  if (flags & ~(SUBDIV_FLAG_REBUILD_EACH_LEVEL | SUBDIV_FLAG_KEEP_STATE)) return SUBDIV_INVALID_ARG;
  // the kept state is that of the carried-over adjacency
  if ((flags & SUBDIV_FLAG_KEEP_STATE) && (rebuilds_levels(scheme, flags) || scheme == SUBDIV_SQRT3_KOBBELT))
    return SUBDIV_INVALID_ARG;
  if (!ws) return SUBDIV_INVALID_ARG;
  hipStream_t s = static_cast<hipStream_t>(stream);
  const long long H0 = cage_H(mesh);
  Sizes L0[SUBDIV_MAX_LEVELS + 1];
  ws_planned(ws, 0);  // the level-0 region is rewritten from here on
  level_sizes(scheme, 0, mesh->num_vertices, mesh->num_faces, H0, H0, H0, 0, 0.f, mesh->num_creases, L0);
  const Layout y0 = make_layout(scheme, 0, flags, L0, mesh->num_creases);
  if (ws_bytes < y0.level0_end) return SUBDIV_WORKSPACE;
  SUBDIV_TRY(init_weight_tables());
  if ((st = plan_enqueue(mesh, scheme, levels, ws, y0, s)) != SUBDIV_OK) return st;
  DeviceInfo hinfo{};
  SUBDIV_TRY(hipMemcpyAsync(&hinfo, at<DeviceInfo>(ws, y0.info), sizeof(hinfo), hipMemcpyDeviceToHost, s));
  SUBDIV_TRY(hipStreamSynchronize(s));
  if ((st = plan_status(hinfo, scheme, levels)) != SUBDIV_OK) return st;
  float max_sharp;
  std::memcpy(&max_sharp, &hinfo.max_sharp_bits, 4);
  if ((st = fill_plan(plan, mesh, scheme, levels, flags, hinfo.num_edges, hinfo.num_boundary, max_sharp,
                      hinfo.max_valence, ws)) != SUBDIV_OK)
    return st;
  ws_planned(ws, plan->priv_stamp);
  return SUBDIV_OK;
}

int subdiv_refine(const subdiv_mesh *mesh, const subdiv_plan_info *plan, subdiv_level_out *outs, void *ws,
                  size_t ws_bytes, void *stream) {
  const int st = refine_impl(mesh, plan, outs, ws, ws_bytes, stream);
  if (st == SUBDIV_HIP) ws_planned(ws, 0);  // part of the work may be missing: the workspace holds nothing usable
  return st;
}

}  // extern "C"

// ---- the library's own workspace, for callers that cannot allocate -------
// A file-scope device array: each GPU the library runs on holds its own copy
// from the load of the code object until the process ends. Host code never
// passes the array's name to a kernel or a copy (on the host it is a
// stand-in, not a device address): the first call on a device, with that
// device current, asks HIP for the array's address there and keeps it.
namespace {
__device__ __align__(256) unsigned char scratch[SUBDIV_STATIC_WORKSPACE_BYTES];

constexpr int kMaxDevices = 64;
std::mutex g_scratch_mu;
void *g_scratch_ptr[kMaxDevices] = {};

int static_workspace(void **out) {
  int dev = -1;
  hipError_t e = hipGetDevice(&dev);
  if (e != hipSuccess) return hip_fail(e);
  if (dev < 0 || dev >= kMaxDevices) return SUBDIV_INVALID_ARG;
  std::lock_guard<std::mutex> lock(g_scratch_mu);
  if (!g_scratch_ptr[dev]) {
    void *ptr = nullptr;
    e = hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch));
    if (e != hipSuccess) return hip_fail(e);
    if (!ptr) return SUBDIV_HIP;
    g_scratch_ptr[dev] = ptr;
  }
  *out = g_scratch_ptr[dev];
  return SUBDIV_OK;
}
}  // namespace

extern "C" {

int subdiv_refine_static(const subdiv_mesh *mesh, const subdiv_plan_info *plan, subdiv_level_out *outs,
                         void *stream) {
  if (!plan || !outs) return SUBDIV_INVALID_ARG;
  // the kept state would live where the caller cannot name it
  if (plan->flags & SUBDIV_FLAG_KEEP_STATE) return SUBDIV_INVALID_ARG;
  if (plan->priv_stamp == 0) return SUBDIV_STATE;
  if (plan->workspace_bytes > SUBDIV_STATIC_WORKSPACE_BYTES) {
    g_last_error = "plan needs " + std::to_string(plan->workspace_bytes) + " workspace bytes; the static workspace holds " +
                   std::to_string((size_t)SUBDIV_STATIC_WORKSPACE_BYTES);
    return SUBDIV_WORKSPACE;
  }
  void *ws = nullptr;
  int st = static_workspace(&ws);
  if (st != SUBDIV_OK) return st;
  st = refine_impl(mesh, plan, outs, ws, SUBDIV_STATIC_WORKSPACE_BYTES, stream);
  if (st == SUBDIV_HIP) ws_planned(ws, 0);
  return st;
}

}  // extern "C"

namespace {
int refine_impl(const subdiv_mesh *mesh, const subdiv_plan_info *plan, subdiv_level_out *outs, void *ws,
                size_t ws_bytes, void *stream) {
  if (!plan || !outs || !ws) return SUBDIV_INVALID_ARG;
  int st = check_mesh_args(mesh, plan->scheme, plan->levels);
  if (st != SUBDIV_OK) return st;
  if (plan->priv_stamp == 0 || mesh->face_verts != plan->priv_mesh_verts) return SUBDIV_STATE;
  const int scheme = plan->scheme, levels = plan->levels;
  if (!outs[levels].face_verts || !outs[levels].positions) return SUBDIV_INVALID_ARG;
  for (int k = 1; k <= levels; ++k)  // face tables are written as int4 rows
    if (reinterpret_cast<uintptr_t>(outs[k].face_verts) % 16 != 0) return SUBDIV_INVALID_ARG;
  if (ws_bytes < plan->workspace_bytes) return SUBDIV_WORKSPACE;
  hipStream_t s = static_cast<hipStream_t>(stream);
  const long long H0 = cage_H(mesh);
  Sizes L[SUBDIV_MAX_LEVELS + 1];
  level_sizes(scheme, levels, mesh->num_vertices, mesh->num_faces, H0, plan->level[0].num_edges,
              plan->level[0].num_boundary_edges, plan->level[0].face_order, plan->max_sharpness, mesh->num_creases,
              L);
  const Layout y = make_layout(scheme, levels, plan->flags, L, mesh->num_creases);
  const bool rebuild = rebuilds_levels(scheme, plan->flags);
  Topo t = cage_topo(mesh, H0, ws, y);
  DeviceInfo *dinfo = at<DeviceInfo>(ws, y.info);
  const bool cr0 = mesh->num_creases > 0;
  Adj a = adj_at(ws, y.adj0, L[0].E, cr0 && L[0].creases);
  const bool keep = (plan->flags & SUBDIV_FLAG_KEEP_STATE) != 0;
  const bool reuse = ws_record(ws).plan == plan->priv_stamp;
  // from here on the workspace holds this plan's level-0 adjacency and, with
  // the state kept, every level's topology once the enqueued work has run
  ws_refined(ws, plan->priv_stamp, keep);
  if (!reuse) {  // the plan's level-0 adjacency is not in this workspace: build it again
    SUBDIV_TIMED("build", 0, build_level0_faces(mesh, scheme, t, ws, y, s));
    BuildScratch b = scratch0(ws, y);
    Adj full = adj_at(ws, y.adj0, H0, cr0);
    SUBDIV_TIMED("build", 0, build_adjacency(t, scheme, b, full, dinfo, s));
    SUBDIV_TIMED("build", 0,
                 build_creases(t, b, full, mesh->num_creases, mesh->crease_verts, mesh->crease_sharpness, dinfo, s));
  }
  bool any_edge_list = false;
  for (int k = 1; k <= levels; ++k) any_edge_list = any_edge_list || outs[k].edge_verts != nullptr;
  // (sqrt(3), with the boundary cycle too, numbers its kept boundary edges by
  // this prefix only for edge ids, which it carries only for edge lists, or
  // with the state kept: its new points are numbered by faces)
  const bool sqrt3_family = scheme == SUBDIV_SQRT3 || scheme == SUBDIV_SQRT3_KOBBELT;
  const bool sqrt3_ids = sqrt3_family && (keep || any_edge_list);
  if (L[0].B > 0 && scheme != SUBDIV_LOOP && (!sqrt3_family || sqrt3_ids)) {
    // boundary prefix: CC edge-point ids, sqrt(3) kept boundary edges
    BuildScratch b = scratch0(ws, y);
    SUBDIV_TIMED("bscan", 0, build_bscan(t, b, a, s));
  }
  const float *P = mesh->positions;
  DeviceInfo *dinfo2 = at<DeviceInfo>(ws, y.info2);
  if (scheme == SUBDIV_CATMULL_CLARK && !rebuild) {
    return refine_cc_carried(mesh, outs, ws, y, L, levels, plan->flags, t, a, P, false, s);
  }
  // ---- generic build of every level (Loop, sqrt(3); Catmull-Clark on request)
  Adj aprev{};  // adjacency of level k-1 (the previous slot, or the cage's)
  Adj aprev2{};  // adjacency of level k-2
  Topo tprev{};  // mesh matrix of level k-1
  bool ep_two_up = false;  // the step before the last wrote final points (Loop: edge points; sqrt(3): face points)
  // The last Loop or sqrt(3) step from level levels-2 (no adjacency of level
  // levels-1): when that level is a refined one and the caller wants no edge
  // list of level levels-1
  // (the last step from level levels-2 has no crease rules; it writes the
  // edge list of level levels-1 itself)
  const bool tri_lag = ::tri_lag(scheme, plan->flags, levels, L);
  const bool lag2 = tri_lag2(scheme, plan->flags, levels, L);
  // level k's adjacency (and face table): a rotating slot, or with the state
  // kept the level's own region
  auto tri_slot = [&](int k) -> const AdjOffsets & { return keep ? y.keep[k] : y.slot[k & 1]; };
  // sqrt(3) old-vertex steps whose neighbours are the face points of level l >= 1:
  // the cage's vertices and face points read their rings from the cage
  auto cage_rings = [&](TriStep &o, int l) {
    if (l < 1) return;
    o.a0 = adj_at(ws, y.adj0, L[0].E, false);
    o.V0 = (int32_t)L[0].V;
    o.F0 = (int32_t)L[0].F;
    int p3 = 1;
    for (int i = 1; i < l; ++i) p3 *= 3;
    o.pow3 = p3;
  };
  for (int k = 0; k < levels; ++k) {
    const bool final = (k == levels - 1);
    int32_t *fv1 = outs[k + 1].face_verts ? outs[k + 1].face_verts : at<int32_t>(ws, y.mfv[(k + 1) & 1]);
    if (keep && scheme != SUBDIV_CATMULL_CLARK && !final) fv1 = at<int32_t>(ws, y.keep[k + 1].fv);
    float *P1 = outs[k + 1].positions ? outs[k + 1].positions : at<float>(ws, y.mP[(k + 1) & 1]);
    if (final) {
      fv1 = outs[k + 1].face_verts;
      P1 = outs[k + 1].positions;
    }
    if (k >= 1 && rebuild) {
      // generic mapped M M^T build of level k (the paper's per-level build)
      BuildScratch b = scratch_rebuild(ws, y);
      Adj slot = adj_at(ws, y.slot[k & 1], L[k].E, L[k].creases);
      SUBDIV_TRY(launch_fill_i32(reinterpret_cast<int32_t *>(dinfo2), 0, sizeof(DeviceInfo) / 4, s));
      SUBDIV_TIMED("rebuild", k, build_faces(t, scheme, b, dinfo2, s));
      SUBDIV_TIMED("rebuild", k, build_adjacency(t, scheme, b, slot, dinfo2, s));
      if (L[k].B > 0 && scheme == SUBDIV_CATMULL_CLARK) SUBDIV_TIMED("bscan", k, build_bscan(t, b, slot, s));
      a = slot;
    }
    const Adj ak = a;
    // (the steps from the level below write the edge list themselves)
    if (outs[k + 1].edge_verts && !(tri_lag && final) && !(lag2 && k == levels - 2))
      SUBDIV_TIMED("edge_export", k, launch_edge_export(t, a, outs[k + 1].edge_verts, s));
    if (scheme == SUBDIV_CATMULL_CLARK) {
      CCStep c{};
      c.t = t;
      c.a = a;
      c.P = P;
      c.fv1 = fv1;
      c.P1 = P1;
      c.has_bnd = L[k].B > 0;
      c.creases = L[k].creases && a.sig != nullptr;
      c.creases1 = L[k + 1].creases != 0;
      // only the inherited sharpness is carried over: the next level is rebuilt
      if (!final) {
        if (c.creases1) c.sig1 = adj_at(ws, y.slot[(k + 1) & 1], L[k + 1].E, true).sig;
      } else if (c.creases1 && outs[k + 1].crease_sharpness) {
        c.sig1 = outs[k + 1].crease_sharpness;
      }
      if (!c.creases) c.sig1 = nullptr;
      SUBDIV_TIMED("cc_face", k, cc_launch(CC_FACE, c, s));
      SUBDIV_TIMED("cc_vertex", k, cc_launch(CC_VERTEX, c, s));
      SUBDIV_TIMED("cc_edge", k, cc_launch(CC_EDGE, c, s));
      if (!final && c.sig1 && outs[k + 1].crease_sharpness)
        SUBDIV_TRY(hipMemcpyAsync(outs[k + 1].crease_sharpness, c.sig1, 8 * L[k + 1].E, hipMemcpyDeviceToDevice,
                                  s));
      a = adj_at(ws, y.slot[(k + 1) & 1], L[k + 1].E, L[k + 1].creases);
    } else if (lag2 && k == levels - 2) {
      // the step before the last, also from the level below (m = k-1, whose
      // adjacency `aprev` and edge or face bases tbase step k-1 left in
      // place): level k's bases (for the last step) into tbase2, counted on
      // level k (sqrt(3): only for the caller's edge list); level k+1's points
      // from level m; its faces only for the caller
      TriStep cnt{t, a, P, nullptr, nullptr, Adj{}, at<int32_t>(ws, y.tbase2), (int32_t)L[k].B};
      if (scheme != SUBDIV_LOOP && outs[levels].edge_verts) {
        SUBDIV_TIMED("sqrt3_count", k, tri_launch(SQRT3_COUNT, cnt, s));
        SUBDIV_TIMED("sqrt3_scan", k, launch_scan(cnt.base, cnt.base, t.F, at<int32_t>(ws, y.partials), nullptr, s));
      }
      TriLag g{tprev, aprev, at<int32_t>(ws, y.tbase), P, (int32_t)L[k].V, (int32_t)L[k].E,
               outs[k + 1].face_verts, P1, outs[k + 1].edge_verts, (int32_t)L[k].B};
      // Loop: level k's edge counts come out of the edge kernel's runs (in
      // closed form from level m) and are scanned after it. The lanes also
      // write the final points of level k's points born on level m (Loop: the
      // edge points; sqrt(3): the face points), unless the final buffer
      // overlaps level k's or level k+1's
      if (scheme == SUBDIV_LOOP) g.cnt1 = cnt.base;
      {
        float *PL = outs[levels].positions;
        auto apart = [&](const float *x, long long nx) { return PL + 3 * L[levels].V <= x || x + nx <= PL; };
        if (apart(P, 3 * L[k].V) && apart(P1, 3 * L[k + 1].V)) {
          g.Pk2 = PL;
          g.vhek = a.vhe;
          ep_two_up = true;
        }
      }
      TriStep o{};  // level m's vertices walk their level-m rings
      o.t = tprev;
      o.P = P;
      o.P1 = P1;
      o.Vg = (int32_t)L[k - 1].V;
      o.ap = aprev;
      o.Vq = (int32_t)L[k - 2].V;
      if (scheme == SUBDIV_SQRT3) cage_rings(o, k - 1);
      if (scheme == SUBDIV_LOOP) {
        SUBDIV_TIMED("loop_vertex", k, tri_launch(LOOP_VERTEX, o, s));
        SUBDIV_TIMED("loop_edge", k, tri_lag_launch(LAG_LOOP_EDGE, g, s));
        SUBDIV_TIMED("loop_scan", k, launch_scan(cnt.base, cnt.base, a.E, at<int32_t>(ws, y.partials), nullptr, s));
        if (g.fv2) SUBDIV_TIMED("loop_face", k, tri_lag_launch(LAG_LOOP_FACE, g, s));
      } else {
        SUBDIV_TIMED("sqrt3_vertex", k, tri_launch(SQRT3_VERTEX, o, s));
        SUBDIV_TIMED("sqrt3_face", k, tri_lag_launch(LAG_SQRT3_FACE, g, s));
      }
    } else if (tri_lag && final) {
      // level k+1 from level m = k-1: `a` and `tprev` are level m's (the step
      // before carried nothing); Loop's edge bases of level m are in tbase
      // (tbase2 when the step before also ran from below)
      const TriLag g{tprev, a, at<int32_t>(ws, lag2 ? y.tbase2 : y.tbase), P, (int32_t)L[k].V, (int32_t)L[k].E,
                     fv1, P1, outs[k + 1].edge_verts, (int32_t)L[k].B};
      TriStep o{};  // the old vertices (level m's) walk their level-m rings
      o.t = tprev;
      o.P = P;
      o.P1 = P1;
      o.Vg = (int32_t)L[k - 1].V;
      o.ap = a;
      o.Vq = (int32_t)L[k - 2].V;
      // level m-1's adjacency is still in place (step k-1 carried nothing):
      // the older vertices walk there
      o.app = aprev2;
      o.Vr = k >= 3 ? (int32_t)L[k - 3].V : 0;
      // level m's vertices born on level m-1 have their points from the step
      // before (sqrt(3): those away from the boundary): only the others walk
      if (ep_two_up && scheme == SUBDIV_LOOP) o.t.V = o.Vq;
      if (ep_two_up && scheme == SUBDIV_SQRT3) o.fp_done = 1;
      if (scheme == SUBDIV_SQRT3) cage_rings(o, k - 1);
      if (scheme == SUBDIV_LOOP) {
        SUBDIV_TIMED("loop_vertex", k, tri_launch(LOOP_VERTEX, o, s));
        SUBDIV_TIMED("loop_edge", k, tri_lag_launch(LAG_LOOP_EDGE, g, s));
        SUBDIV_TIMED("loop_face", k, tri_lag_launch(LAG_LOOP_FACE, g, s));
      } else {
        SUBDIV_TIMED("sqrt3_vertex", k, tri_launch(SQRT3_VERTEX, o, s));
        SUBDIV_TIMED("sqrt3_face", k, tri_lag_launch(LAG_SQRT3_FACE, g, s));
      }
    } else if (scheme == SUBDIV_SQRT3_KOBBELT && k % 2 == 1) {
      // the trisection step of the boundary cycle (level k came from a sqrt(3) step)
      TrisectStep ts{t, a, P, fv1, P1, at<int32_t>(ws, y.tslot), at<int32_t>(ws, y.trank),
                     at<int32_t>(ws, y.tnb)};
      const bool carry = !rebuild && !final;  // level k+1's adjacency in closed form
      if (carry) {
        ts.a1 = adj_at(ws, tri_slot(k + 1), L[k + 1].E, false);
        if (sqrt3_ids) {
          ts.base = at<int32_t>(ws, y.tbase3);
          ts.pmask = at<uint8_t>(ws, y.tmask);
          ts.nbnd = (int32_t)L[k].B;
        } else {  // twins and ring starts alone (see the sqrt(3) step)
          ts.a1.eid = ts.a1.e2h = ts.a1.bscan = nullptr;
        }
      }
      ts.fpV = (int32_t)L[k - 1].V;  // (k is odd: level k was refined from level k-1)
      ts.fpF = (int32_t)L[k - 1].F;
      // level k-1's adjacency stays in place until this step's face kernel
      // (the per-level build walks level k instead, the form this is checked against)
      if (!rebuild) ts.ap = aprev;
      SUBDIV_TIMED("sqrt3_trisect", k, trisect_launch(TRISECT_MARK, ts, s));
      SUBDIV_TIMED("sqrt3_trisect", k, launch_scan(ts.brank, ts.brank, t.F, at<int32_t>(ws, y.partials), nullptr, s));
      if (carry && sqrt3_ids) {
        SUBDIV_TIMED("sqrt3_trisect", k, trisect_launch(TRISECT_COUNT, ts, s));
        SUBDIV_TIMED("sqrt3_trisect", k,
                     launch_scan(ts.base, ts.base, 2ll * t.F, at<int32_t>(ws, y.partials), nullptr, s));
      }
      // (the vertex step writes the old vertices' starts that the face step may lower)
      SUBDIV_TIMED("sqrt3_trisect", k, trisect_launch(TRISECT_VERTEX, ts, s));
      SUBDIV_TIMED("sqrt3_trisect", k, trisect_launch(TRISECT_FACE, ts, s));
      if (carry) a = ts.a1;
    } else {
      // (sqrt(3) with the boundary cycle: a level after a trisection step has
      // boundary points among its new vertices, so the vertex step walks the
      // rings on the level itself; the points born from faces away from the
      // boundary read theirs from their child rows)
      const bool walk_own = scheme == SUBDIV_SQRT3_KOBBELT;
      TriStep c{t, a, P, fv1, P1, Adj{}, nullptr, (int32_t)L[k].B, (k >= 1 && !walk_own) ? (int32_t)L[k - 1].V : 0,
                aprev, k >= 2 ? (int32_t)L[k - 2].V : 0};
      if (walk_own && k >= 1) {  // the points born from level k-1's faces
        c.fpV = (int32_t)L[k - 1].V;
        c.fpF = (int32_t)L[k - 1].F;
        // a level made by the trisection step (the step before was one): its
        // old vertices' rings from level k-1's fans and boundary slots, which
        // stay in place until this step's face kernel (the per-level build
        // walks them on level k, the form the closed one is checked against)
        if (k % 2 == 0 && !rebuild) {
          c.pbslot = at<int32_t>(ws, y.tslot);
          c.pbrank = at<int32_t>(ws, y.trank);
        }
      }
      // before the last step from level k: Loop still needs level k's edge
      // bases; nothing is carried, and level k+1's face table is only written
      // for the caller
      const bool before_lag = tri_lag && k == levels - 2;
      const bool carry = !rebuild && !final && !before_lag;  // level k+1's adjacency in closed form
      // Loop creases of level k, and whether level k+1 inherits any
      const bool lcr = scheme == SUBDIV_LOOP && L[k].creases && a.sig && a.vcr;
      double *sig1 = nullptr;
      if (lcr && L[k + 1].creases)
        sig1 = final ? outs[k + 1].crease_sharpness : adj_at(ws, tri_slot(k + 1), L[k + 1].E, true).sig;
      // sqrt(3): the edge ids of a level (and the face bases of the level
      // before, which number them) are read only to number the next level's
      // edges and for edge lists; with no edge list asked for, carry the
      // twins and ring starts alone
      const bool twins_only = carry && sqrt3_family && !sqrt3_ids;
      if (carry) {
        c.a1 = adj_at(ws, tri_slot(k + 1), L[k + 1].E, L[k + 1].creases != 0);
        c.a1.bscan = nullptr;  // sqrt(3): the boundary edges of a refined level are its first ids
        if (twins_only) c.a1.eid = c.a1.e2h = nullptr;
      }
      if ((carry && !twins_only) || (before_lag && scheme == SUBDIV_LOOP) || sig1) c.base = at<int32_t>(ws, y.tbase);
      if (before_lag && !outs[k + 1].face_verts) c.fv1 = nullptr;
      if (scheme == SUBDIV_LOOP) {
        SUBDIV_TIMED("loop_edge", k, tri_launch(LOOP_EDGE, c, s));
        if (c.base)
          SUBDIV_TIMED("loop_scan", k, launch_scan(c.base, c.base, a.E, at<int32_t>(ws, y.partials), nullptr, s));
        // the vertex step walks level k-1's adjacency, whose slot the carried
        // face step overwrites with level k+1's: it runs first
        SUBDIV_TIMED("loop_vertex", k, tri_launch(LOOP_VERTEX, c, s));
        if (c.fv1) SUBDIV_TIMED("loop_face", k, tri_launch(LOOP_FACE, c, s));
        if (lcr) {
          if (sig1) SUBDIV_TRY(launch_fill_i32(reinterpret_cast<int32_t *>(sig1), 0, 2 * L[k + 1].E, s));
          SUBDIV_TIMED("loop_crease", k, loop_crease_launch(c, sig1, s));
          if (!final && sig1 && outs[k + 1].crease_sharpness)
            SUBDIV_TRY(hipMemcpyAsync(outs[k + 1].crease_sharpness, sig1, 8 * L[k + 1].E, hipMemcpyDeviceToDevice, s));
        }
        if (carry) a = c.a1;
      } else {
        // (before the last step from level k with an edge list asked for, the
        // face bases of level k give that list's ids)
        if (before_lag && outs[levels].edge_verts) c.base = at<int32_t>(ws, y.tbase);
        if (c.base) {
          SUBDIV_TIMED("sqrt3_count", k, tri_launch(SQRT3_COUNT, c, s));
          SUBDIV_TIMED("sqrt3_scan", k, launch_scan(c.base, c.base, t.F, at<int32_t>(ws, y.partials), nullptr, s));
        }
        // the vertex step reads level k-1's adjacency, whose slot the carried
        // face step overwrites with level k+1's: it runs first
        SUBDIV_TIMED("sqrt3_vertex", k, tri_launch(SQRT3_VERTEX, c, s));
        SUBDIV_TIMED("sqrt3_face", k, tri_launch(SQRT3_FACE, c, s));
        if (carry) a = c.a1;
      }
    }
    if (keep && scheme != SUBDIV_CATMULL_CLARK && !final && outs[k + 1].face_verts)
      SUBDIV_TRY(hipMemcpyAsync(outs[k + 1].face_verts, fv1, 4 * L[k + 1].H, hipMemcpyDeviceToDevice, s));
    // level k+1 becomes the input of the next step
    tprev = t;
    aprev2 = aprev;
    t = Topo{(int32_t)L[k + 1].V, (int32_t)L[k + 1].F, (int32_t)L[k + 1].H, L[k + 1].order, nullptr, nullptr, fv1};
    P = P1;
    aprev = ak;
  }
  return SUBDIV_OK;
}
}  // namespace

extern "C" {

int subdiv_refine_positions(const subdiv_mesh *mesh, const subdiv_plan_info *plan, subdiv_level_out *outs,
                            void *ws, size_t ws_bytes, void *stream) {
  if (!plan || !outs || !ws) return SUBDIV_INVALID_ARG;
  int st = check_mesh_args(mesh, plan->scheme, plan->levels);
  if (st != SUBDIV_OK) return st;
  if (plan->priv_stamp == 0 || mesh->face_verts != plan->priv_mesh_verts || !state_kept(plan, ws))
    return SUBDIV_STATE;
  if (!(plan->flags & SUBDIV_FLAG_KEEP_STATE)) return SUBDIV_STATE;
  const int levels = plan->levels;
  if (!outs[levels].positions) return SUBDIV_INVALID_ARG;
  if (ws_bytes < plan->workspace_bytes) return SUBDIV_WORKSPACE;
  hipStream_t s = static_cast<hipStream_t>(stream);
  const long long H0 = cage_H(mesh);
  Sizes L[SUBDIV_MAX_LEVELS + 1];
  level_sizes(plan->scheme, levels, mesh->num_vertices, mesh->num_faces, H0, plan->level[0].num_edges,
              plan->level[0].num_boundary_edges, plan->level[0].face_order, plan->max_sharpness, mesh->num_creases,
              L);
  const Layout y = make_layout(plan->scheme, levels, plan->flags, L, mesh->num_creases);
  const Topo t = cage_topo(mesh, H0, ws, y);
  const Adj a = adj_at(ws, y.adj0, L[0].E, mesh->num_creases > 0 && L[0].creases);
  if (plan->scheme != SUBDIV_CATMULL_CLARK) return refine_tri_kept(plan->scheme, outs, ws, y, L, levels, t, a, mesh->positions, s);
  return refine_cc_carried(mesh, outs, ws, y, L, levels, plan->flags, t, a, mesh->positions, true, s);
}

int subdiv_refine_vertex_data(const subdiv_mesh *mesh, const subdiv_plan_info *plan, const float *data, int dim,
                              float *out, void *ws, size_t ws_bytes, void *stream) {
  if (!plan || !data || !out || !ws || dim < 1) return SUBDIV_INVALID_ARG;
  int st = check_mesh_args(mesh, plan->scheme, plan->levels);
  if (st != SUBDIV_OK) return st;
  if (plan->priv_stamp == 0 || mesh->face_verts != plan->priv_mesh_verts || !state_kept(plan, ws))
    return SUBDIV_STATE;
  if (!(plan->flags & SUBDIV_FLAG_KEEP_STATE)) return SUBDIV_STATE;
  if (ws_bytes < plan->workspace_bytes) return SUBDIV_WORKSPACE;
  hipStream_t s = static_cast<hipStream_t>(stream);
  const int levels = plan->levels;
  const long long H0 = cage_H(mesh);
  Sizes L[SUBDIV_MAX_LEVELS + 1];
  level_sizes(plan->scheme, levels, mesh->num_vertices, mesh->num_faces, H0, plan->level[0].num_edges,
              plan->level[0].num_boundary_edges, plan->level[0].face_order, plan->max_sharpness, mesh->num_creases,
              L);
  const Layout y = make_layout(plan->scheme, levels, plan->flags, L, mesh->num_creases);
  const Topo t = cage_topo(mesh, H0, ws, y);
  const Adj a = adj_at(ws, y.adj0, L[0].E, mesh->num_creases > 0 && L[0].creases);
  // Scratch of the adjoint: its term buffer ([max_k H_k * 3] >= [V_0 * 3])
  // carries the cage slice, its two gradient buffers (each [max_k V_k * 3])
  // the final slices of two groups of three channels; the levels in between
  // use the usual buffers. Six channels at a time are then written into out
  // by one kernel, whole rows when dim <= 6.
  float *slice0 = at<float>(ws, y.bterm);
  float *sliceL[2] = {at<float>(ws, y.bg[0]), at<float>(ws, y.bg[1])};
  subdiv_mesh m = *mesh;
  m.positions = slice0;
  subdiv_level_out outs[SUBDIV_MAX_LEVELS + 1] = {};
  for (int c0 = 0; c0 < dim; c0 += 6) {
    for (int g = 0; g < 2 && c0 + 3 * g < dim; ++g) {
      SUBDIV_TRY(launch_pack3(data, dim, c0 + 3 * g, L[0].V, slice0, s));
      outs[levels].positions = sliceL[g];
      st = plan->scheme == SUBDIV_CATMULL_CLARK
               ? refine_cc_carried(&m, outs, ws, y, L, levels, plan->flags, t, a, slice0, true, s)
               : refine_tri_kept(plan->scheme, outs, ws, y, L, levels, t, a, slice0, s);
      if (st != SUBDIV_OK) return st;
    }
    const int ncols = dim - c0 < 6 ? dim - c0 : 6;
    SUBDIV_TRY(launch_unpack6(sliceL[0], sliceL[1], dim, c0, ncols, L[levels].V, out, s));
  }
  return SUBDIV_OK;
}

int subdiv_select(const subdiv_mesh *mesh, const subdiv_plan_info *plan, const uint8_t *seed, int rings, void *ws,
                  size_t ws_bytes, subdiv_selection *sel, void *stream) {
  return subdiv_select_ex(mesh, plan, seed, rings, 0u, ws, ws_bytes, sel, stream);
}

int subdiv_select_ex(const subdiv_mesh *mesh, const subdiv_plan_info *plan, const uint8_t *seed, int rings,
                     uint32_t flags, void *ws, size_t ws_bytes, subdiv_selection *sel, void *stream) {
  if (!sel) return SUBDIV_INVALID_ARG;
  std::memset(sel, 0, sizeof(*sel));
  if (!plan || !ws || !mesh || rings < 1 || (flags & ~SUBDIV_SELECT_CLOSE_PINCHES)) return SUBDIV_INVALID_ARG;
  if (plan->priv_stamp == 0 || mesh->face_verts != plan->priv_mesh_verts || ws != plan->priv_ws ||
      ws_record(ws).plan != plan->priv_stamp)
    return SUBDIV_STATE;
  int st = check_mesh_args(mesh, plan->scheme, plan->levels);
  if (st != SUBDIV_OK) return st;
  if (ws_bytes < plan->workspace_bytes) return SUBDIV_WORKSPACE;
  hipStream_t s = static_cast<hipStream_t>(stream);
  const long long H0 = cage_H(mesh);
  Sizes L[SUBDIV_MAX_LEVELS + 1];
  level_sizes(plan->scheme, plan->levels, mesh->num_vertices, mesh->num_faces, H0, plan->level[0].num_edges,
              plan->level[0].num_boundary_edges, plan->level[0].face_order, plan->max_sharpness, mesh->num_creases,
              L);
  const Layout y = make_layout(plan->scheme, plan->levels, plan->flags, L, mesh->num_creases);
  const Topo t = cage_topo(mesh, H0, ws, y);
  const Adj a = adj_at(ws, y.adj0, L[0].E, mesh->num_creases > 0);
  const SelectScratch w = select_scratch(ws, y);
  const bool close = (flags & SUBDIV_SELECT_CLOSE_PINCHES) != 0;
  SUBDIV_TRY(select_region(t, a, w, seed, at<int32_t>(ws, y.nval), rings, close, s));
  int32_t tot[4], last = 0;
  SUBDIV_TRY(hipMemcpyAsync(tot, w.totals, sizeof(tot), hipMemcpyDeviceToHost, s));
  if (close) SUBDIV_TRY(hipMemcpyAsync(&last, w.changed + kPinchPasses - 1, 4, hipMemcpyDeviceToHost, s));
  SUBDIV_TRY(hipStreamSynchronize(s));
  if (last) return SUBDIV_NONMANIFOLD;  // still pinched after every pass
  sel->num_vertices = tot[0];
  sel->num_faces = tot[1];
  sel->num_halfedges = t.order > 0 ? tot[1] * t.order : tot[2];
  sel->num_creases = tot[3];
  sel->face_order = t.order;
  sel->rings = rings;
  sel->flags = flags;
  sel->priv_stamp = plan->priv_stamp;
  sel->priv_ws = ws;
  return SUBDIV_OK;
}

int subdiv_extract(const subdiv_mesh *mesh, const subdiv_plan_info *plan, const subdiv_selection *sel,
                   const subdiv_extraction *out, void *ws, size_t ws_bytes, void *stream) {
  if (!plan || !sel || !out || !ws || !mesh) return SUBDIV_INVALID_ARG;
  if (plan->priv_stamp == 0 || mesh->face_verts != plan->priv_mesh_verts || ws != plan->priv_ws ||
      ws_record(ws).plan != plan->priv_stamp || sel->priv_stamp != plan->priv_stamp || sel->priv_ws != ws)
    return SUBDIV_STATE;
  int st = check_mesh_args(mesh, plan->scheme, plan->levels);
  if (st != SUBDIV_OK) return st;
  if (ws_bytes < plan->workspace_bytes) return SUBDIV_WORKSPACE;
  if (sel->num_vertices == 0) return SUBDIV_OK;
  if (!out->face_verts || !out->positions || (sel->face_order == 0 && !out->face_offsets) ||
      (sel->num_creases > 0 && (!out->crease_verts || !out->crease_sharpness)))
    return SUBDIV_INVALID_ARG;
  hipStream_t s = static_cast<hipStream_t>(stream);
  const long long H0 = cage_H(mesh);
  Sizes L[SUBDIV_MAX_LEVELS + 1];
  level_sizes(plan->scheme, plan->levels, mesh->num_vertices, mesh->num_faces, H0, plan->level[0].num_edges,
              plan->level[0].num_boundary_edges, plan->level[0].face_order, plan->max_sharpness, mesh->num_creases,
              L);
  const Layout y = make_layout(plan->scheme, plan->levels, plan->flags, L, mesh->num_creases);
  const Topo t = cage_topo(mesh, H0, ws, y);
  const Adj a = adj_at(ws, y.adj0, L[0].E, mesh->num_creases > 0);
  ExtractOut o{out->seed_flags, out->face_verts, out->face_offsets, out->face_map, out->vertex_map,
               out->crease_verts, out->positions, out->crease_sharpness, sel->num_faces, sel->num_creases};
  SUBDIV_TRY(extract_region(t, a, select_scratch(ws, y), sel->rings, mesh->positions, o, s));
  return SUBDIV_OK;
}

}  // extern "C"

namespace {
// The adjoint's view of level k of a kept state: topology, adjacency, the
// parent level's sizes for the closed-form classes, and the coefficients.
BwdStep bwd_level(const subdiv_mesh *mesh, void *ws, const Layout &y, const Sizes *L, long long H0, int k) {
  BwdStep b{};
  if (k == 0) {
    b.t = cage_topo(mesh, H0, ws, y);
    b.a = adj_at(ws, y.adj0, L[0].E, mesh->num_creases > 0 && L[0].creases);
  } else {
    b.a = adj_at(ws, y.keep[k], L[k].E, L[k].creases);
    b.t = Topo{(int32_t)L[k].V, (int32_t)L[k].F, (int32_t)L[k].H, 4, nullptr, nullptr, b.a.fv};
  }
  if (k >= 2) {  // level k-1 is all quads
    const Adj ap = adj_at(ws, y.keep[k - 1], L[k - 1].E, false);
    b.Vp = (int32_t)L[k - 1].V;
    b.Fp = (int32_t)L[k - 1].F;
    b.bscan_p = L[k - 1].B > 0 ? ap.bscan : nullptr;
  }
  b.coef = at<float>(ws, y.kcoef[k]);
  return b;
}

// (the coefficients of a plan are computed on its first backward pass)
int keep_bw_coefs(const subdiv_mesh *mesh, void *ws, const Layout &y, const Sizes *L, int levels, hipStream_t s) {
  const long long H0 = cage_H(mesh);
  for (int k = 0; k < levels; ++k) {
    const BwdStep b = bwd_level(mesh, ws, y, L, H0, k);
    SUBDIV_TIMED("bw_coef", k, bw_launch(BW_COEF, b, s));
  }
  return SUBDIV_OK;
}
}  // namespace

extern "C" {

int subdiv_backward(const subdiv_mesh *mesh, const subdiv_plan_info *plan, const float *grad_out, float *grad_in,
                    void *ws, size_t ws_bytes, void *stream) {
  if (!plan || !grad_out || !grad_in || !ws) return SUBDIV_INVALID_ARG;
  int st = check_mesh_args(mesh, plan->scheme, plan->levels);
  if (st != SUBDIV_OK) return st;
  if (plan->priv_stamp == 0 || mesh->face_verts != plan->priv_mesh_verts) return SUBDIV_STATE;
  if (!(plan->flags & SUBDIV_FLAG_KEEP_STATE) || !state_kept(plan, ws)) return SUBDIV_STATE;
  if (plan->scheme != SUBDIV_CATMULL_CLARK) return SUBDIV_STATE;  // the adjoint covers Catmull-Clark
  if (ws_bytes < plan->workspace_bytes) return SUBDIV_WORKSPACE;
  hipStream_t s = static_cast<hipStream_t>(stream);
  const int levels = plan->levels;
  const long long H0 = cage_H(mesh);
  Sizes L[SUBDIV_MAX_LEVELS + 1];
  level_sizes(plan->scheme, levels, mesh->num_vertices, mesh->num_faces, H0, plan->level[0].num_edges,
              plan->level[0].num_boundary_edges, plan->level[0].face_order, plan->max_sharpness, mesh->num_creases,
              L);
  const Layout y = make_layout(plan->scheme, levels, plan->flags, L, mesh->num_creases);
  if (ws_record(ws).coef != plan->priv_stamp) {
    if ((st = keep_bw_coefs(mesh, ws, y, L, levels, s)) != SUBDIV_OK) return st;
    ws_coefs(ws, plan->priv_stamp);
  }
  const float *g1 = grad_out;
  for (int k = levels - 1; k >= 0; --k) {
    BwdStep b = bwd_level(mesh, ws, y, L, H0, k);  // the plan's kept coefficients
    b.g1 = g1;
    b.g0 = (k == 0) ? grad_in : at<float>(ws, y.bg[k & 1]);
    b.term = at<float>(ws, y.bterm);
    SUBDIV_TIMED("bw_face", k, bw_launch(BW_FACE, b, s));
    SUBDIV_TIMED("bw_vertex", k, bw_launch(BW_VERTEX, b, s));
    g1 = b.g0;
  }
  return SUBDIV_OK;
}

int subdiv_state_destroy(const subdiv_plan_info *plan, const void *ws) {
  if (!plan || !ws) return SUBDIV_INVALID_ARG;
  std::lock_guard<std::mutex> lock(g_ws_mu);
  const auto it = g_ws.find(ws);
  if (plan->priv_stamp == 0 || it == g_ws.end() ||
      (it->second.plan != plan->priv_stamp && it->second.kept != plan->priv_stamp))
    return SUBDIV_STATE;
  g_ws.erase(it);
  return SUBDIV_OK;
}

}  // extern "C"

// ---- batches ------------------------------------------------------------
// A batch lists meshes with a scheme and a level count each. Its meshes are
// grouped by (scheme, levels), in order of first appearance; the members of
// a group keep their batch order. A group of several meshes is packed into
// one disjoint union cage and refined by the ordinary kernels, one launch per
// stage for the whole group; a group of one is the mesh itself.
namespace {

struct Group {
  int scheme = 0, levels = 0;
  std::vector<int> idx;  // batch indices of the members
  long long VU = 0, FU = 0, HU = 0, CU = 0;
  int order = 0;
  bool general = false;
  Sizes L[SUBDIV_MAX_LEVELS + 1];  // sizes of the union's levels (exact when the members' counts are known)
  size_t desc = 0, tables = 0, outtab = 0, stats = 0, ufv = 0, uoff = 0, uP = 0, ucv = 0, ucs = 0, fvL = 0, PL = 0;
  size_t uws = 0, uws_bytes = 0;
  bool single() const { return idx.size() == 1; }
};

std::vector<Group> make_groups(const int *schemes, const int *levels, int n) {
  std::vector<Group> g;
  for (int i = 0; i < n; ++i) {
    size_t k = 0;
    for (; k < g.size(); ++k)
      if (g[k].scheme == schemes[i] && g[k].levels == levels[i]) break;
    if (k == g.size()) {
      g.emplace_back();
      g.back().scheme = schemes[i];
      g.back().levels = levels[i];
    }
    g[k].idx.push_back(i);
  }
  return g;
}

// blocks of the union's final vertex ids: V_0, then per level F_k and/or E_k
int gather_blocks(int scheme, int levels) { return 1 + levels * (scheme == SUBDIV_CATMULL_CLARK ? 2 : 1); }

// Sizes and workspace regions of every group. for_plan: the symbolic pass
// (the union cage, per-member statistics and the level-0 region); otherwise
// the refinement (cages, gather tables, the union's final level and the
// union's whole workspace). plans: the members' counts (edges, boundary
// edges, largest sharpness), or nullptr for the upper bound E, B <= H.
bool layout_groups(std::vector<Group> &gs, const subdiv_mesh *m, const subdiv_plan_info *plans, uint32_t flags,
                   bool for_plan, size_t *total) {
  const long long lim = 0x7fffffffLL - 16;
  Carver c;
  for (Group &g : gs) {
    long long EU = 0, BU = 0;
    float smax = 0.f;
    g.VU = g.FU = g.HU = g.CU = 0;
    g.order = m[g.idx[0]].face_offsets ? 0 : m[g.idx[0]].face_order;
    for (const int i : g.idx) {
      g.VU += m[i].num_vertices;
      g.FU += m[i].num_faces;
      g.HU += cage_H(&m[i]);
      g.CU += m[i].num_creases;
      const int oi = m[i].face_offsets ? 0 : m[i].face_order;
      if (oi != g.order) g.order = 0;
      if (plans) {
        EU += plans[i].level[0].num_edges;
        BU += plans[i].level[0].num_boundary_edges;
        smax = plans[i].max_sharpness > smax ? plans[i].max_sharpness : smax;
      }
    }
    if (g.VU > lim || g.FU > lim || g.HU > lim || g.CU > lim) return false;
    if (!plans) {
      EU = BU = g.HU;
      smax = g.CU > 0 ? 1e30f : 0.f;
    }
    g.general = (g.order == 0);
    const int lv = for_plan ? 0 : g.levels;
    level_sizes(g.scheme, lv, g.VU, g.FU, g.HU, EU, BU, g.order, smax, g.CU, g.L);
    if (!sizes_fit_int32(g.L, lv)) return false;
    const Layout y = make_layout(g.scheme, lv, flags, g.L, g.CU);
    g.uws_bytes = for_plan ? y.level0_end : y.total;
    const size_t n = g.idx.size();
    if (!g.single()) {
      g.desc = c.take(sizeof(BatchMesh) * n);
      if (for_plan) {
        g.stats = c.take(4 * (4 * n + 1));  // edge prefix [n+1], boundary, valence and sharpness maxima [n] each
      } else {
        const size_t nblk = (size_t)gather_blocks(g.scheme, g.levels), nseg = nblk * n;
        g.tables = c.take(16 * nseg + 4 * (nseg + 1 + nblk + 1 + nseg + 2 * (n + 1)));
        g.outtab = c.take(sizeof(BatchOut) * n);
        g.uP = c.take(12 * g.VU);
        g.fvL = c.take(4 * g.L[g.levels].H);
        g.PL = c.take(12 * g.L[g.levels].V);
      }
      g.ufv = c.take(4 * g.HU);
      g.uoff = g.general ? c.take(4 * (g.FU + 1)) : 0;
      g.ucv = c.take(8 * (g.CU > 0 ? g.CU : 1));
      g.ucs = c.take(4 * (g.CU > 0 ? g.CU : 1));
    }
    g.uws = c.take(g.uws_bytes);
  }
  *total = c.at + 256;
  return true;
}

std::vector<BatchMesh> batch_descriptors(const subdiv_mesh *m, const Group &g) {
  std::vector<BatchMesh> d(g.idx.size());
  int vo = 0, fo = 0, ho = 0, co = 0;
  for (size_t k = 0; k < g.idx.size(); ++k) {
    const subdiv_mesh &x0 = m[g.idx[k]];
    BatchMesh &x = d[k];
    x.fv = x0.face_verts;
    x.off = x0.face_offsets;
    x.order = x0.face_offsets ? 0 : x0.face_order;
    x.P = x0.positions;
    x.cv = x0.crease_verts;
    x.cs = x0.crease_sharpness;
    x.V = x0.num_vertices;
    x.F = x0.num_faces;
    x.H = (int32_t)cage_H(&x0);
    x.C = x0.num_creases;
    x.vofs = vo;
    x.fofs = fo;
    x.hofs = ho;
    x.cofs = co;
    vo += x.V;
    fo += x.F;
    ho += x.H;
    co += x.C;
  }
  return d;
}

subdiv_mesh union_mesh(const Group &g, void *ws) {
  subdiv_mesh u{};
  u.num_vertices = (int32_t)g.VU;
  u.num_faces = (int32_t)g.FU;
  u.face_order = g.general ? 0 : g.order;
  u.num_halfedges = (int32_t)g.HU;
  u.face_offsets = g.general ? at<int32_t>(ws, g.uoff) : nullptr;
  u.face_verts = at<int32_t>(ws, g.ufv);
  u.positions = g.uP ? at<float>(ws, g.uP) : nullptr;
  u.num_creases = (int32_t)g.CU;
  u.crease_verts = g.CU ? at<int32_t>(ws, g.ucv) : nullptr;
  u.crease_sharpness = g.CU ? at<float>(ws, g.ucs) : nullptr;
  return u;
}

// Library-owned pinned staging for the per-call pointer tables of a batch:
// a ring of slots, each reused only after the copy that used it completed.
struct PinnedRing {
  struct Slot {
    void *host = nullptr;
    size_t cap = 0;
    hipEvent_t ev = nullptr;
    bool pending = false;
  };
  std::mutex mu;
  Slot slots[8];
  unsigned next = 0;
};
PinnedRing g_ring;

hipError_t staged_upload(void *dst, const void *src, size_t bytes, hipStream_t s) {
  std::lock_guard<std::mutex> lock(g_ring.mu);
  PinnedRing::Slot &sl = g_ring.slots[g_ring.next++ % 8];
  hipError_t err;
  if (sl.pending && (err = hipEventSynchronize(sl.ev)) != hipSuccess) return err;
  sl.pending = false;
  if (sl.cap < bytes) {
    if (sl.host && (err = hipHostFree(sl.host)) != hipSuccess) return err;
    sl.host = nullptr;
    sl.cap = 0;
    const size_t cap = bytes < 65536 ? 65536 : bytes;
    if ((err = hipHostMalloc(&sl.host, cap, hipHostMallocDefault)) != hipSuccess) return err;
    sl.cap = cap;
  }
  if (!sl.ev && (err = hipEventCreateWithFlags(&sl.ev, hipEventDisableTiming)) != hipSuccess) return err;
  std::memcpy(sl.host, src, bytes);
  if ((err = hipMemcpyAsync(dst, sl.host, bytes, hipMemcpyHostToDevice, s)) != hipSuccess) return err;
  if ((err = hipEventRecord(sl.ev, s)) != hipSuccess) return err;
  sl.pending = true;
  return hipSuccess;
}

int check_batch_args(const subdiv_mesh *m, const int *schemes, const int *levels, int n) {
  if (!m || !schemes || !levels || n < 1 || n > SUBDIV_MAX_BATCH) return SUBDIV_INVALID_ARG;
  for (int i = 0; i < n; ++i) {
    const int st = check_mesh_args(&m[i], schemes[i], levels[i]);
    if (st != SUBDIV_OK) return st;
    if (m[i].num_creases > 0 && schemes[i] != SUBDIV_CATMULL_CLARK) return SUBDIV_INVALID_ARG;  // batches: CC creases
    if (schemes[i] == SUBDIV_SQRT3_KOBBELT) return SUBDIV_INVALID_ARG;  // not in batches
  }
  return SUBDIV_OK;
}

// a member's plan may serve this batch entry: same cage, scheme, and at least
// as many levels validated
bool member_plan_ok(const subdiv_plan_info &p, const subdiv_mesh &m, int scheme, int levels) {
  return p.priv_stamp != 0 && p.priv_mesh_verts == m.face_verts && p.scheme == scheme && p.levels >= levels &&
         !(p.flags & SUBDIV_FLAG_KEEP_STATE) && p.level[0].num_vertices == m.num_vertices &&
         p.level[0].num_faces == m.num_faces && p.level[0].num_halfedges == cage_H(&m);
}

// The final gather of a group: block b of the union's level-L vertex ids
// lists the members in order; member k numbers its vertices by its segments
// of the blocks in block order. LS[k] are member k's level sizes.
struct GatherPlan {
  std::vector<int32_t> tab;
  int face_chunks = 0, vertex_chunks = 0, nblk = 0;
};

bool gather_plan(const Group &g, const std::vector<Sizes> &LS, GatherPlan &gp) {
  const int n = (int)g.idx.size(), levels = g.levels;
  const bool has_f = g.scheme != SUBDIV_LOOP, has_e = g.scheme != SUBDIV_SQRT3;
  const int per = (int)has_f + (int)has_e;
  const int nblk = gather_blocks(g.scheme, levels), nseg = nblk * n;
  auto bsize = [&](int blk, int k) -> long long {
    const Sizes *Li = &LS[(size_t)k * (levels + 1)];
    if (blk == 0) return Li[0].V;
    const int lev = (blk - 1) / per, t = (blk - 1) % per;
    return (has_f && t == 0) ? Li[lev].F : Li[lev].E;
  };
  std::vector<int32_t> seg(4 * (size_t)nseg), pch((size_t)nseg + 1, 0), ub((size_t)nblk + 1, 0), doff((size_t)nseg),
      fpre((size_t)n + 1, 0), fch((size_t)n + 1, 0);
  std::vector<long long> loc((size_t)n, 0);
  for (int blk = 0; blk < nblk; ++blk) {
    long long pre = 0;
    for (int k = 0; k < n; ++k) {
      const long long len = bsize(blk, k), x = blk * (long long)n + k;
      seg[4 * x + 0] = (int32_t)(ub[blk] + pre);
      seg[4 * x + 1] = k;
      seg[4 * x + 2] = (int32_t)loc[k];
      seg[4 * x + 3] = (int32_t)len;
      doff[x] = (int32_t)(loc[k] - ub[blk] - pre);
      pch[x + 1] = pch[x] + (int32_t)((len + kGather - 1) / kGather);
      loc[k] += len;
      pre += len;
    }
    ub[blk + 1] = (int32_t)(ub[blk] + pre);
  }
  for (int k = 0; k < n; ++k) {
    const long long FLk = LS[(size_t)k * (levels + 1) + levels].F;
    fpre[k + 1] = fpre[k] + (int32_t)FLk;
    fch[k + 1] = fch[k] + (int32_t)((FLk + kGather - 1) / kGather);
  }
  if (ub[nblk] != g.L[levels].V || fpre[n] != g.L[levels].F) return false;
  gp.tab.clear();
  for (const auto *v : {&seg, &pch, &ub, &doff, &fpre, &fch}) gp.tab.insert(gp.tab.end(), v->begin(), v->end());
  gp.face_chunks = fch[n];
  gp.vertex_chunks = pch[nseg];
  gp.nblk = nblk;
  return true;
}

}  // namespace

extern "C" {

size_t subdiv_batch_workspace_bound(const subdiv_mesh *meshes, const int *schemes, const int *levels, int n,
                                    const subdiv_plan_info *plans, uint32_t flags) {
  if (check_batch_args(meshes, schemes, levels, n) != SUBDIV_OK) return 0;
  if (flags & ~SUBDIV_FLAG_REBUILD_EACH_LEVEL) return 0;
  if (plans)
    for (int i = 0; i < n; ++i)
      if (!member_plan_ok(plans[i], meshes[i], schemes[i], levels[i])) return 0;
  std::vector<Group> gs = make_groups(schemes, levels, n);
  size_t need_plan = 0, need_refine = 0;
  if (!layout_groups(gs, meshes, nullptr, flags, true, &need_plan)) return 0;
  if (!layout_groups(gs, meshes, plans, flags, false, &need_refine)) return 0;
  return need_plan > need_refine ? need_plan : need_refine;
}

int subdiv_plan_batch(const subdiv_mesh *meshes, const int *schemes, const int *levels, int n, uint32_t flags,
                      void *ws, size_t ws_bytes, subdiv_plan_info *plans, void *stream) {
  if (!plans || !ws) return SUBDIV_INVALID_ARG;
  int st = check_batch_args(meshes, schemes, levels, n);
  if (st != SUBDIV_OK) return st;
  for (int i = 0; i < n; ++i) std::memset(&plans[i], 0, sizeof(plans[i]));
  if (flags & ~SUBDIV_FLAG_REBUILD_EACH_LEVEL) return SUBDIV_INVALID_ARG;
  std::vector<Group> gs = make_groups(schemes, levels, n);
  size_t need = 0;
  if (!layout_groups(gs, meshes, nullptr, flags, true, &need)) return SUBDIV_INVALID_ARG;
  if (ws_bytes < need) return SUBDIV_WORKSPACE;
  hipStream_t s = static_cast<hipStream_t>(stream);
  ws_forget_range(ws, ws_bytes);
  SUBDIV_TRY(init_weight_tables());
  // every group's symbolic pass is enqueued before the one read-back
  for (const Group &g : gs) {
    void *uws = at<void>(ws, g.uws);
    if (g.single()) {
      const int i = g.idx[0];
      Sizes L0[SUBDIV_MAX_LEVELS + 1];
      level_sizes(g.scheme, 0, g.VU, g.FU, g.HU, g.HU, g.HU, 0, 0.f, g.CU, L0);
      if ((st = plan_enqueue(&meshes[i], g.scheme, g.levels, uws, make_layout(g.scheme, 0, flags, L0, g.CU), s)) !=
          SUBDIV_OK)
        return st;
      continue;
    }
    const std::vector<BatchMesh> desc = batch_descriptors(meshes, g);
    const int ng = (int)g.idx.size();
    SUBDIV_TRY(staged_upload(at<void>(ws, g.desc), desc.data(), sizeof(BatchMesh) * desc.size(), s));
    const BatchUnion u{at<int32_t>(ws, g.ufv), g.general ? at<int32_t>(ws, g.uoff) : nullptr, at<int32_t>(ws, g.ucv),
                       at<float>(ws, g.ucs)};
    long long items = g.HU;
    items = (g.FU + 1 > items) ? g.FU + 1 : items;
    items = (g.CU > items) ? g.CU : items;
    SUBDIV_TRY(batch_concat_topology(at<BatchMesh>(ws, g.desc), ng, u, items, s));
    const subdiv_mesh um = union_mesh(g, ws);
    const Layout y0 = make_layout(g.scheme, 0, flags, g.L, g.CU);
    if ((st = plan_enqueue(&um, g.scheme, g.levels, uws, y0, s)) != SUBDIV_OK) return st;
    // per-member edge and boundary counts and maxima, from the union's build
    int32_t *stats = at<int32_t>(ws, g.stats);
    SUBDIV_TRY(batch_stats(at<BatchMesh>(ws, g.desc), ng, at<int32_t>(uws, y0.ebase), at<int32_t>(uws, y0.bflag),
                           at<int32_t>(uws, y0.rowptr), g.CU ? at<float>(ws, g.ucs) : nullptr, g.VU, g.HU, g.CU, stats,
                           stats + ng + 1, stats + 2 * ng + 1, stats + 3 * ng + 1, s));
  }
  std::vector<DeviceInfo> hinfo(gs.size());
  std::vector<std::vector<int32_t>> hstats(gs.size());
  for (size_t k = 0; k < gs.size(); ++k) {
    const Group &g = gs[k];
    void *uws = at<void>(ws, g.uws);
    Sizes L0[SUBDIV_MAX_LEVELS + 1];
    level_sizes(g.scheme, 0, g.VU, g.FU, g.HU, g.HU, g.HU, 0, 0.f, g.CU, L0);
    const Layout y0 = make_layout(g.scheme, 0, flags, L0, g.CU);
    SUBDIV_TRY(hipMemcpyAsync(&hinfo[k], at<DeviceInfo>(uws, y0.info), sizeof(DeviceInfo), hipMemcpyDeviceToHost, s));
    if (!g.single()) {
      hstats[k].resize(4 * g.idx.size() + 1);
      SUBDIV_TRY(hipMemcpyAsync(hstats[k].data(), at<int32_t>(ws, g.stats), 4 * hstats[k].size(),
                                hipMemcpyDeviceToHost, s));
    }
  }
  SUBDIV_TRY(hipStreamSynchronize(s));
  for (size_t k = 0; k < gs.size(); ++k)
    if ((st = plan_status(hinfo[k], gs[k].scheme, gs[k].levels)) != SUBDIV_OK) return st;
  for (size_t k = 0; k < gs.size(); ++k) {
    const Group &g = gs[k];
    const int ng = (int)g.idx.size();
    for (int j = 0; j < ng; ++j) {
      const int i = g.idx[j];
      long long E0, B0;
      int vmax;
      float smax;
      if (g.single()) {
        E0 = hinfo[k].num_edges;
        B0 = hinfo[k].num_boundary;
        vmax = hinfo[k].max_valence;
        std::memcpy(&smax, &hinfo[k].max_sharp_bits, 4);
      } else {
        const int32_t *h = hstats[k].data();
        E0 = h[j + 1] - h[j];
        B0 = h[ng + 1 + j];
        vmax = h[2 * ng + 1 + j];
        std::memcpy(&smax, &h[3 * ng + 1 + j], 4);
      }
      if (meshes[i].num_creases == 0) smax = 0.f;
      if ((st = fill_plan(&plans[i], &meshes[i], g.scheme, g.levels, flags, E0, B0, smax, vmax, nullptr)) !=
          SUBDIV_OK)
        return st;
    }
  }
  ws_forget_range(ws, ws_bytes);
  return SUBDIV_OK;
}

int subdiv_refine_batch(const subdiv_mesh *meshes, const int *schemes, const int *levels, int n,
                        const subdiv_plan_info *plans, subdiv_level_out *outs, void *ws, size_t ws_bytes,
                        void *stream) {
  if (!plans || !outs || !ws) return SUBDIV_INVALID_ARG;
  int st = check_batch_args(meshes, schemes, levels, n);
  if (st != SUBDIV_OK) return st;
  for (int i = 0; i < n; ++i) {
    if (!member_plan_ok(plans[i], meshes[i], schemes[i], levels[i])) return SUBDIV_STATE;
    if (!outs[i].face_verts || !outs[i].positions || reinterpret_cast<uintptr_t>(outs[i].face_verts) % 16 != 0)
      return SUBDIV_INVALID_ARG;
  }
  const uint32_t flags = plans[0].flags & SUBDIV_FLAG_REBUILD_EACH_LEVEL;
  std::vector<Group> gs = make_groups(schemes, levels, n);
  size_t need = 0;
  if (!layout_groups(gs, meshes, plans, flags, false, &need)) return SUBDIV_INVALID_ARG;
  if (ws_bytes < need) return SUBDIV_WORKSPACE;
  hipStream_t s = static_cast<hipStream_t>(stream);
  ws_forget_range(ws, ws_bytes);
  SUBDIV_TRY(init_weight_tables());
  for (const Group &g : gs) {
    const int L = g.levels, ng = (int)g.idx.size();
    void *uws = at<void>(ws, g.uws);
    // every member's sizes for its level count (its plan may cover more levels)
    std::vector<Sizes> LS((size_t)ng * (L + 1));
    for (int j = 0; j < ng; ++j) {
      const subdiv_plan_info &p = plans[g.idx[j]];
      const subdiv_mesh &mj = meshes[g.idx[j]];
      level_sizes(g.scheme, L, mj.num_vertices, mj.num_faces, cage_H(&mj), p.level[0].num_edges,
                  p.level[0].num_boundary_edges, mj.face_offsets ? 0 : mj.face_order, p.max_sharpness, mj.num_creases,
                  &LS[(size_t)j * (L + 1)]);
    }
    if (g.single()) {
      // the mesh itself, straight into its outputs, with its plan for this level count
      const int i = g.idx[0];
      subdiv_plan_info p;
      if ((st = fill_plan(&p, &meshes[i], g.scheme, L, flags, plans[i].level[0].num_edges,
                          plans[i].level[0].num_boundary_edges, plans[i].max_sharpness, plans[i].max_valence,
                          nullptr)) != SUBDIV_OK)
        return st;
      subdiv_level_out uo[SUBDIV_MAX_LEVELS + 1] = {};
      uo[L].face_verts = outs[i].face_verts;
      uo[L].positions = outs[i].positions;
      if ((st = refine_impl(&meshes[i], &p, uo, uws, g.uws_bytes, s)) != SUBDIV_OK) return st;
      continue;
    }
    const std::vector<BatchMesh> desc = batch_descriptors(meshes, g);
    std::vector<BatchOut> ot((size_t)ng);
    for (int j = 0; j < ng; ++j) ot[j] = BatchOut{outs[g.idx[j]].face_verts, outs[g.idx[j]].positions};
    GatherPlan gp;
    if (!gather_plan(g, LS, gp)) return SUBDIV_STATE;
    SUBDIV_TRY(staged_upload(at<void>(ws, g.desc), desc.data(), sizeof(BatchMesh) * desc.size(), s));
    SUBDIV_TRY(staged_upload(at<void>(ws, g.outtab), ot.data(), sizeof(BatchOut) * ot.size(), s));
    SUBDIV_TRY(staged_upload(at<void>(ws, g.tables), gp.tab.data(), 4 * gp.tab.size(), s));
    const BatchUnion u{at<int32_t>(ws, g.ufv), g.general ? at<int32_t>(ws, g.uoff) : nullptr, at<int32_t>(ws, g.ucv),
                       at<float>(ws, g.ucs)};
    long long items = g.HU;
    items = (g.FU + 1 > items) ? g.FU + 1 : items;
    items = (g.CU > items) ? g.CU : items;
    SUBDIV_TRY(batch_concat_topology(at<BatchMesh>(ws, g.desc), ng, u, items, s));
    SUBDIV_TRY(batch_concat_positions(at<BatchMesh>(ws, g.desc), ng, at<float>(ws, g.uP), g.VU, s));
    // the union's plan from its members' counts (a disjoint union of valid
    // cages is valid); refine_impl builds its cage adjacency in uws
    const subdiv_mesh um = union_mesh(g, ws);
    float smax = 0.f;
    int vmax = 0;
    for (const int i : g.idx) {
      smax = plans[i].max_sharpness > smax ? plans[i].max_sharpness : smax;
      vmax = plans[i].max_valence > vmax ? plans[i].max_valence : vmax;
    }
    subdiv_plan_info up;
    if ((st = fill_plan(&up, &um, g.scheme, L, flags, g.L[0].E, g.L[0].B, smax, vmax, nullptr)) != SUBDIV_OK)
      return st;
    subdiv_level_out uo[SUBDIV_MAX_LEVELS + 1] = {};
    uo[L].face_verts = at<int32_t>(ws, g.fvL);
    uo[L].positions = at<float>(ws, g.PL);
    if ((st = refine_impl(&um, &up, uo, uws, g.uws_bytes, s)) != SUBDIV_OK) return st;
    BatchTables t{};
    t.n = ng;
    t.order = g.scheme == SUBDIV_CATMULL_CLARK ? 4 : 3;
    t.nblk = gp.nblk;
    t.nseg = t.nblk * ng;
    const int32_t *tb = at<int32_t>(ws, g.tables);
    t.seg = reinterpret_cast<const int4 *>(tb);
    t.pch = tb + 4ll * t.nseg;
    t.ub = t.pch + t.nseg + 1;
    t.doff = t.ub + t.nblk + 1;
    t.fpre = t.doff + t.nseg;
    t.fch = t.fpre + ng + 1;
    SUBDIV_TIMED("batch_extract", L,
                 batch_extract(t, at<int32_t>(ws, g.fvL), at<float>(ws, g.PL), at<BatchOut>(ws, g.outtab),
                               gp.face_chunks, gp.vertex_chunks, s));
  }
  return SUBDIV_OK;
}

}  // extern "C"
