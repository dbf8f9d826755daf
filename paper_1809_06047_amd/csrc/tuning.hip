// Launch-shape table of libsubdiv: the workgroup size of each tunable kernel
// per size bucket, as measured by the tuner (paper_1809_06047_amd/tune.py)
// on gfx950 and committed as JSON beside the library.
//
// Table format (other top-level keys are ignored):
//   {"kernels": {"lag2_group": [[max_items, block], ...], ...}}
// Per kernel, entries are ordered by max_items; an element count n takes the
// first entry with n <= max_items, an entry with max_items < 0 takes every
// count, and a count past the last entry takes the last one. Blocks are 64,
// 128, 256 or 512. A kernel absent from the table runs with 256.
//
// The table is read once, at the library's first launch: from the path in
// the environment variable SUBDIV_TUNING when it is set (empty: none), else
// from tuning_gfx950.json next to libsubdiv.so when that file exists.
// subdiv_tuning_load replaces it at any time.
#include <dlfcn.h>

#include <atomic>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <mutex>
#include <string>
#include <vector>

#include "subdiv_internal.h"

namespace subdiv {

namespace {

const char *const kKeyNames[TK_COUNT] = {
    "lag_group",  "lag_vertex",  "lag_edge",    "lag2_group",  "lag2_combine", "lag2_older",
    "loop_edge",  "loop_vertex", "loop_face",   "sqrt3_count", "sqrt3_face",   "sqrt3_vertex",
    "loopl_face", "loopl_edge",  "sqrt3l_face", "bw_coef",     "bw_face",      "bw_vertex"};

struct Entry {
  long long max_items;  // < 0: no bound
  int block;
};
using Table = std::vector<Entry>[TK_COUNT];

std::mutex g_mu;
Table g_table;
std::string g_source = "built-in";
bool g_loaded = false;  // the default table was looked for (or a table was set)

thread_local int tl_key = -1;
thread_local long long tl_items = 0;
thread_local int tl_block = 0;

bool valid_block(long long b) { return b == 64 || b == 128 || b == 256 || b == 512; }

int key_of(const char *name) {
  for (int k = 0; k < TK_COUNT; ++k)
    if (std::strcmp(name, kKeyNames[k]) == 0) return k;
  return -1;
}

// ---- a small JSON reader: enough to walk any document and to read the
// "kernels" object of arrays of integer pairs
struct Json {
  const char *p, *end;
  std::string err;

  void ws() {
    while (p < end && (*p == ' ' || *p == '\n' || *p == '\r' || *p == '\t')) ++p;
  }
  bool expect(char c) {
    ws();
    if (p < end && *p == c) {
      ++p;
      return true;
    }
    if (err.empty()) err = std::string("expected '") + c + "'";
    return false;
  }
  bool peek(char c) {
    ws();
    return p < end && *p == c;
  }
  bool string(std::string &out) {
    if (!expect('"')) return false;
    out.clear();
    while (p < end && *p != '"') {
      if (*p == '\\') {
        if (++p >= end) break;
        if (*p == 'u') {  // keep the escape as text: keys and names here are ASCII
          if (end - p < 5) break;
          out += "\\u";
          out.append(p + 1, 4);
          p += 5;
          continue;
        }
        const char c = *p == 'n' ? '\n' : *p == 't' ? '\t' : *p == 'r' ? '\r' : *p == 'b' ? '\b' : *p == 'f' ? '\f' : *p;
        out += c;
        ++p;
        continue;
      }
      out += *p++;
    }
    if (p >= end) {
      err = "unterminated string";
      return false;
    }
    ++p;
    return true;
  }
  bool integer(long long &v) {
    ws();
    char *e = nullptr;
    const long long x = std::strtoll(p, &e, 10);
    if (e == p || (e < end && (*e == '.' || *e == 'e' || *e == 'E'))) {
      err = "expected an integer";
      return false;
    }
    v = x;
    p = e;
    return true;
  }
  bool skip() {  // any value
    ws();
    if (p >= end) {
      err = "unexpected end";
      return false;
    }
    if (*p == '"') {
      std::string s;
      return string(s);
    }
    if (*p == '{' || *p == '[') {
      const char close = *p == '{' ? '}' : ']';
      const bool obj = *p == '{';
      ++p;
      if (peek(close)) {
        ++p;
        return true;
      }
      while (true) {
        if (obj) {
          std::string k;
          if (!string(k) || !expect(':')) return false;
        }
        if (!skip()) return false;
        if (peek(',')) {
          ++p;
          continue;
        }
        return expect(close);
      }
    }
    const char *s = p;
    while (p < end && (std::strchr("+-.eE", *p) || (*p >= '0' && *p <= '9') || (*p >= 'a' && *p <= 'z'))) ++p;
    if (p == s) {
      err = "unexpected character";
      return false;
    }
    return true;
  }
  // [[max_items, block], ...]
  bool entries(std::vector<Entry> &out) {
    if (!expect('[')) return false;
    out.clear();
    if (peek(']')) {
      ++p;
      return true;
    }
    while (true) {
      long long m, b;
      if (!expect('[') || !integer(m) || !expect(',') || !integer(b) || !expect(']')) return false;
      if (!valid_block(b)) {
        err = "block " + std::to_string(b) + " is not 64, 128, 256 or 512";
        return false;
      }
      out.push_back(Entry{m, (int)b});
      if (peek(',')) {
        ++p;
        continue;
      }
      return expect(']');
    }
  }
  bool document(Table &t) {
    if (!expect('{')) return false;
    if (peek('}')) {
      ++p;
      return true;
    }
    while (true) {
      std::string key;
      if (!string(key) || !expect(':')) return false;
      if (key == "kernels") {
        if (!expect('{')) return false;
        if (!peek('}')) {
          while (true) {
            std::string name;
            if (!string(name) || !expect(':')) return false;
            const int k = key_of(name.c_str());
            if (k < 0) {
              err = "unknown kernel \"" + name + "\"";
              return false;
            }
            if (!entries(t[k])) return false;
            if (peek(',')) {
              ++p;
              continue;
            }
            break;
          }
        }
        if (!expect('}')) return false;
      } else if (!skip()) {
        return false;
      }
      if (peek(',')) {
        ++p;
        continue;
      }
      return expect('}');
    }
  }
};

// entries ordered by their bound, the unbounded one last
bool ordered(const std::vector<Entry> &v) {
  for (size_t i = 0; i + 1 < v.size(); ++i) {
    if (v[i].max_items < 0) return false;
    if (v[i + 1].max_items >= 0 && v[i + 1].max_items <= v[i].max_items) return false;
  }
  return true;
}

int load_file(const char *path, std::string &why) {
  FILE *f = std::fopen(path, "rb");
  if (!f) {
    why = std::string("cannot open ") + path;
    return SUBDIV_INVALID_ARG;
  }
  std::string text;
  char buf[4096];
  size_t n;
  while ((n = std::fread(buf, 1, sizeof(buf), f)) > 0) text.append(buf, n);
  std::fclose(f);
  Table t;
  Json j{text.data(), text.data() + text.size(), {}};
  if (!j.document(t)) {
    why = std::string(path) + ": " + j.err;
    return SUBDIV_INVALID_ARG;
  }
  for (int k = 0; k < TK_COUNT; ++k)
    if (!ordered(t[k])) {
      why = std::string(path) + ": entries of " + kKeyNames[k] + " are not ordered by max_items";
      return SUBDIV_INVALID_ARG;
    }
  for (int k = 0; k < TK_COUNT; ++k) g_table[k] = t[k];
  g_source = path;
  return SUBDIV_OK;
}

// the default table, looked for once (g_mu held)
void ensure_loaded() {
  if (g_loaded) return;
  g_loaded = true;
  std::string path;
  if (const char *env = std::getenv("SUBDIV_TUNING")) {
    path = env;
  } else {
    Dl_info info{};
    if (dladdr(reinterpret_cast<const void *>(&tune_key_name), &info) && info.dli_fname) {
      path = info.dli_fname;
      const size_t slash = path.rfind('/');
      path = (slash == std::string::npos ? std::string(".") : path.substr(0, slash)) + "/tuning_gfx950.json";
      FILE *f = std::fopen(path.c_str(), "rb");
      if (!f) path.clear();
      else std::fclose(f);
    }
  }
  if (path.empty()) return;
  std::string why;
  if (load_file(path.c_str(), why) != SUBDIV_OK) g_source = "built-in (" + why + ")";
}

int lookup(int key, long long items) {
  const std::vector<Entry> &v = g_table[key];
  if (v.empty()) return kBlock;
  for (const Entry &e : v)
    if (e.max_items < 0 || items <= e.max_items) return e.block;
  return v.back().block;
}

}  // namespace

const char *tune_key_name(int key) { return key >= 0 && key < TK_COUNT ? kKeyNames[key] : "?"; }

int tuned_block(int key, long long items) {
  int b;
  {
    std::lock_guard<std::mutex> lock(g_mu);
    ensure_loaded();
    b = lookup(key, items);
  }
  tl_key = key;
  tl_items = items;
  tl_block = b;
  return b;
}

void tune_note_reset() { tl_key = -1; }

bool tune_note_take(int *key, long long *items, int *block) {
  if (tl_key < 0) return false;
  *key = tl_key;
  *items = tl_items;
  *block = tl_block;
  tl_key = -1;
  return true;
}

}  // namespace subdiv

using namespace subdiv;

extern "C" {

int subdiv_tuning_load(const char *path) {
  std::lock_guard<std::mutex> lock(g_mu);
  g_loaded = true;
  if (!path || !*path) {
    for (auto &v : g_table) v.clear();
    g_source = "built-in";
    return SUBDIV_OK;
  }
  std::string why;
  const int st = load_file(path, why);
  if (st != SUBDIV_OK) subdiv_set_error(why.c_str());
  return st;
}

int subdiv_tuning_set(const char *kernel, int64_t max_items, int block) {
  if (!kernel || !valid_block(block)) return SUBDIV_INVALID_ARG;
  const bool all = std::strcmp(kernel, "*") == 0;
  const int k = all ? -1 : key_of(kernel);
  if (!all && k < 0) return SUBDIV_INVALID_ARG;
  std::lock_guard<std::mutex> lock(g_mu);
  ensure_loaded();
  for (int i = 0; i < TK_COUNT; ++i) {
    if (!all && i != k) continue;
    std::vector<Entry> &v = g_table[i];
    if (max_items < 0) {
      v.assign(1, Entry{-1, block});
      continue;
    }
    bool done = false;
    for (Entry &e : v)
      if (e.max_items == max_items) {
        e.block = block;
        done = true;
      }
    if (!done) {
      size_t at = 0;
      while (at < v.size() && v[at].max_items >= 0 && v[at].max_items < max_items) ++at;
      v.insert(v.begin() + at, Entry{max_items, block});
    }
  }
  g_source = "set by subdiv_tuning_set";
  return SUBDIV_OK;
}

int subdiv_tuning_block(const char *kernel, int64_t items) {
  if (!kernel) return SUBDIV_INVALID_ARG;
  const int k = key_of(kernel);
  if (k < 0 || items < 0) return SUBDIV_INVALID_ARG;
  std::lock_guard<std::mutex> lock(g_mu);
  ensure_loaded();
  return lookup(k, items);
}

const char *subdiv_tuning_source(void) {
  std::lock_guard<std::mutex> lock(g_mu);
  ensure_loaded();
  return g_source.c_str();
}

int subdiv_tuning_kernel_name(int index, char *out, int max_out) {
  if (index < 0 || index >= TK_COUNT || !out || max_out < 1) return SUBDIV_INVALID_ARG;
  std::strncpy(out, kKeyNames[index], (size_t)max_out - 1);
  out[max_out - 1] = 0;
  return SUBDIV_OK;
}

}  // extern "C"
