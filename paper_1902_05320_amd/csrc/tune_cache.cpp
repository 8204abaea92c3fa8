// The autotuner's cache: tuned tiles in a JSON file, looked up by the batch
// entry points when the environment variable KBATCH_TUNE names the file.
//
// File format (written by keccak_tune_store, read by keccak_tune_lookup):
//
//   {"format": "kbatch-tune-1",
//    "entries": [
//      {"arch": "gfx950", "rocm": "7.2", "variant": "sha3_256", "batch_class": 24,
//       "nb_class": "*", "waves_per_simd": 3, "steps_per_item": 4, "staging": 2, "ms": 1.7},
//      {"arch": "gfx950", "rocm": "7.2", "variant": "sha3_256", "batch_class": 24,
//       "nb_class": 3, "steps": 8, "threads_per_state": 1},
//      ...]}
//
// Every knob is keyed by what it depends on.  The knobs the host applies
// when it launches (resident waves per SIMD, the staging form, the default
// steps per queue item) are chosen once per launch, so their entries carry
// nb_class "*": one per (arch, ROCm, variant, batch class).  The knobs the
// device applies per bucket of equal block counts (steps per queue item and
// threads per state) carry the block-count class of the bucket, so a launch
// over a batch that spans several classes takes each class's own choice.
//
// batch_class = floor(log2(n)); nb_class = floor(log2(blocks)), capped at
// KB_NB_CLASSES - 1 (blocks = floor(L / R) + 1 of a message).
#include <hip/hip_runtime.h>

#include <cctype>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <map>
#include <memory>
#include <mutex>
#include <string>
#include <sys/stat.h>
#include <vector>

#include "kb_internal.h"
#include "kbatch.h"

namespace {

// ---- a small JSON reader and writer (objects, arrays, strings, numbers) ----

struct JVal {
  enum Kind { kNull, kNum, kStr, kArr, kObj, kBool } kind = kNull;
  double num = 0;
  bool b = false;
  std::string str;
  std::vector<JVal> arr;
  std::vector<std::pair<std::string, JVal>> obj;
  const JVal* get(const char* k) const {
    for (auto& kv : obj)
      if (kv.first == k) return &kv.second;
    return nullptr;
  }
};

struct JParser {
  const char* p;
  const char* end;
  bool ok = true;
  void ws() {
    while (p < end && std::isspace(static_cast<unsigned char>(*p))) ++p;
  }
  bool lit(const char* s) {
    const size_t n = std::strlen(s);
    if (static_cast<size_t>(end - p) >= n && std::strncmp(p, s, n) == 0) {
      p += n;
      return true;
    }
    return false;
  }
  bool string(std::string& out) {
    if (p >= end || *p != '"') return false;
    ++p;
    while (p < end && *p != '"') {
      char c = *p++;
      if (c == '\\') {
        if (p >= end) return false;
        const char e = *p++;
        switch (e) {
          case 'n': c = '\n'; break;
          case 't': c = '\t'; break;
          case 'r': c = '\r'; break;
          case 'b': c = '\b'; break;
          case 'f': c = '\f'; break;
          case 'u':  // keys and values here are ASCII; keep the code point's low byte
            if (end - p < 4) return false;
            c = static_cast<char>(std::strtol(std::string(p, 4).c_str(), nullptr, 16) & 0x7F);
            p += 4;
            break;
          default: c = e;
        }
      }
      out.push_back(c);
    }
    if (p >= end) return false;
    ++p;
    return true;
  }
  bool value(JVal& v, int depth) {
    if (depth > 16) return false;
    ws();
    if (p >= end) return false;
    if (*p == '{') {
      ++p;
      v.kind = JVal::kObj;
      ws();
      if (p < end && *p == '}') {
        ++p;
        return true;
      }
      for (;;) {
        ws();
        std::string k;
        if (!string(k)) return false;
        ws();
        if (p >= end || *p != ':') return false;
        ++p;
        JVal x;
        if (!value(x, depth + 1)) return false;
        v.obj.emplace_back(std::move(k), std::move(x));
        ws();
        if (p < end && *p == ',') {
          ++p;
          continue;
        }
        if (p < end && *p == '}') {
          ++p;
          return true;
        }
        return false;
      }
    }
    if (*p == '[') {
      ++p;
      v.kind = JVal::kArr;
      ws();
      if (p < end && *p == ']') {
        ++p;
        return true;
      }
      for (;;) {
        JVal x;
        if (!value(x, depth + 1)) return false;
        v.arr.push_back(std::move(x));
        ws();
        if (p < end && *p == ',') {
          ++p;
          continue;
        }
        if (p < end && *p == ']') {
          ++p;
          return true;
        }
        return false;
      }
    }
    if (*p == '"') {
      v.kind = JVal::kStr;
      return string(v.str);
    }
    if (lit("null")) return true;
    if (lit("true")) {
      v.kind = JVal::kBool;
      v.b = true;
      return true;
    }
    if (lit("false")) {
      v.kind = JVal::kBool;
      return true;
    }
    char* q = nullptr;
    const std::string tok(p, static_cast<size_t>(end - p < 64 ? end - p : 64));
    v.num = std::strtod(tok.c_str(), &q);
    if (q == tok.c_str()) return false;
    v.kind = JVal::kNum;
    p += q - tok.c_str();
    return true;
  }
};

bool parse_json(const std::string& text, JVal& out) {
  JParser ps{text.data(), text.data() + text.size()};
  if (!ps.value(out, 0)) return false;
  ps.ws();
  return ps.p == ps.end;
}

void write_json_string(std::string& o, const std::string& s) {
  o.push_back('"');
  for (char c : s) {
    if (c == '"' || c == '\\') {
      o.push_back('\\');
      o.push_back(c);
    } else if (static_cast<unsigned char>(c) < 0x20) {
      char buf[8];
      std::snprintf(buf, sizeof buf, "\\u%04x", c);
      o += buf;
    } else {
      o.push_back(c);
    }
  }
  o.push_back('"');
}

// ---- entries ----

struct Entry {
  std::string arch, rocm, variant;
  int batch_class = -1;
  int nb_class = -1;  // -1 = "*": the launch-wide knobs
  // launch-wide
  int waves_per_simd = 0, steps_per_item = 0, staging = 0;
  // per block-count class
  int steps = 0, threads_per_state = 0;
  double ms = -1.0;
  bool same_key(const Entry& e) const {
    return arch == e.arch && rocm == e.rocm && variant == e.variant &&
           batch_class == e.batch_class && nb_class == e.nb_class;
  }
};

int num_or(const JVal& o, const char* k, int dflt) {
  const JVal* v = o.get(k);
  return v && v->kind == JVal::kNum ? static_cast<int>(v->num) : dflt;
}

std::string str_or(const JVal& o, const char* k) {
  const JVal* v = o.get(k);
  return v && v->kind == JVal::kStr ? v->str : std::string();
}

bool read_file(const char* path, std::string& out) {
  FILE* f = std::fopen(path, "rb");
  if (!f) return false;
  char buf[65536];
  size_t r;
  while ((r = std::fread(buf, 1, sizeof buf, f)) > 0) out.append(buf, r);
  std::fclose(f);
  return true;
}

// Parse a cache file.  A missing file is an empty cache; a malformed one is
// an error (KB_EINVAL) so that a typo never silently drops tuned tiles.
int load_entries(const char* path, std::vector<Entry>& out) {
  out.clear();
  std::string text;
  if (!read_file(path, text)) return KB_OK;
  JVal root;
  if (!parse_json(text, root) || root.kind != JVal::kObj)
    return kb::set_last_error(KB_EINVAL, "tune cache: not a JSON object");
  const JVal* fmt = root.get("format");
  if (!fmt || fmt->kind != JVal::kStr || fmt->str != "kbatch-tune-1")
    return kb::set_last_error(KB_EINVAL, "tune cache: format is not kbatch-tune-1");
  const JVal* es = root.get("entries");
  if (!es || es->kind != JVal::kArr) return kb::set_last_error(KB_EINVAL, "tune cache: no entries array");
  for (const JVal& o : es->arr) {
    if (o.kind != JVal::kObj) return kb::set_last_error(KB_EINVAL, "tune cache: entry is not an object");
    Entry e;
    e.arch = str_or(o, "arch");
    e.rocm = str_or(o, "rocm");
    e.variant = str_or(o, "variant");
    e.batch_class = num_or(o, "batch_class", -1);
    const JVal* nc = o.get("nb_class");
    e.nb_class = nc && nc->kind == JVal::kNum ? static_cast<int>(nc->num) : -1;
    e.waves_per_simd = num_or(o, "waves_per_simd", 0);
    e.steps_per_item = num_or(o, "steps_per_item", 0);
    e.staging = num_or(o, "staging", 0);
    e.steps = num_or(o, "steps", 0);
    e.threads_per_state = num_or(o, "threads_per_state", 0);
    const JVal* ms = o.get("ms");
    e.ms = ms && ms->kind == JVal::kNum ? ms->num : -1.0;
    if (e.arch.empty() || e.variant.empty() || e.batch_class < 0 || e.nb_class >= KB_NB_CLASSES)
      return kb::set_last_error(KB_EINVAL, "tune cache: entry lacks arch, variant or batch_class");
    out.push_back(e);
  }
  return KB_OK;
}

int save_entries(const char* path, const std::vector<Entry>& es) {
  std::string o = "{\"format\": \"kbatch-tune-1\",\n \"entries\": [";
  for (size_t k = 0; k < es.size(); ++k) {
    const Entry& e = es[k];
    o += k ? ",\n  {" : "\n  {";
    o += "\"arch\": ";
    write_json_string(o, e.arch);
    o += ", \"rocm\": ";
    write_json_string(o, e.rocm);
    o += ", \"variant\": ";
    write_json_string(o, e.variant);
    char buf[256];
    std::snprintf(buf, sizeof buf, ", \"batch_class\": %d", e.batch_class);
    o += buf;
    if (e.nb_class < 0) {
      std::snprintf(buf, sizeof buf,
                    ", \"nb_class\": \"*\", \"waves_per_simd\": %d, \"steps_per_item\": %d, "
                    "\"staging\": %d",
                    e.waves_per_simd, e.steps_per_item, e.staging);
    } else {
      std::snprintf(buf, sizeof buf, ", \"nb_class\": %d, \"steps\": %d, \"threads_per_state\": %d",
                    e.nb_class, e.steps, e.threads_per_state);
    }
    o += buf;
    if (e.ms >= 0) {
      std::snprintf(buf, sizeof buf, ", \"ms\": %.6g", e.ms);
      o += buf;
    }
    o += "}";
  }
  o += "\n]}\n";
  const std::string tmp = std::string(path) + ".tmp";
  FILE* f = std::fopen(tmp.c_str(), "wb");
  if (!f) return kb::set_last_error(KB_EINVAL, "tune cache: cannot write the file");
  const bool w = std::fwrite(o.data(), 1, o.size(), f) == o.size();
  const bool c = std::fclose(f) == 0;
  if (!w || !c || std::rename(tmp.c_str(), path) != 0) {
    std::remove(tmp.c_str());
    return kb::set_last_error(KB_EINVAL, "tune cache: cannot write the file");
  }
  return KB_OK;
}

const char* variant_name(int v) {
  switch (v) {
    case 0: return "sha3_224";
    case 1: return "sha3_256";
    case 2: return "sha3_384";
    case 3: return "sha3_512";
    case -1: return "mixed";
    default: return nullptr;
  }
}

int floor_log2(uint64_t x) {
  int r = -1;
  while (x) {
    x >>= 1;
    ++r;
  }
  return r;
}

// The current device's architecture name (without target features) and the
// HIP runtime's version as "major.minor".
int device_key(std::string& arch, std::string& rocm) {
  int dev = 0;
  if (hipGetDevice(&dev) != hipSuccess) return kb::set_last_error(KB_EHIP, "hipGetDevice failed");
  hipDeviceProp_t prop;
  if (hipGetDeviceProperties(&prop, dev) != hipSuccess)
    return kb::set_last_error(KB_EHIP, "hipGetDeviceProperties failed");
  arch = prop.gcnArchName;
  const size_t colon = arch.find(':');
  if (colon != std::string::npos) arch.resize(colon);
  int ver = 0;
  if (hipRuntimeGetVersion(&ver) != hipSuccess) return kb::set_last_error(KB_EHIP, "hipRuntimeGetVersion failed");
  char buf[32];
  std::snprintf(buf, sizeof buf, "%d.%d", ver / 10000000, (ver / 100000) % 100);
  rocm = buf;
  return KB_OK;
}

// The (arch, rocm) key: both given, or both NULL for the current device.
int resolve_key(const char* arch_in, const char* rocm_in, std::string& arch, std::string& rocm) {
  if (arch_in && rocm_in) {
    arch = arch_in;
    rocm = rocm_in;
    return KB_OK;
  }
  if (arch_in || rocm_in) return kb::set_last_error(KB_EINVAL, "give both arch and rocm, or neither");
  return device_key(arch, rocm);
}

// Cache of the file named by KBATCH_TUNE, reloaded when its size or
// modification time changes.
struct Loaded {
  std::string path;
  long long mtime = -1, size = -1;
  std::vector<Entry> entries;
  int status = KB_OK;
};
std::mutex g_tmu;
Loaded g_loaded;

int entries_for(const char* path, std::vector<Entry>& out) {
  struct stat st;
  const bool exists = ::stat(path, &st) == 0;
  const long long mt = exists ? static_cast<long long>(st.st_mtim.tv_sec) * 1000000000ll + st.st_mtim.tv_nsec : -1;
  const long long sz = exists ? static_cast<long long>(st.st_size) : -1;
  std::lock_guard<std::mutex> lk(g_tmu);
  if (g_loaded.path != path || g_loaded.mtime != mt || g_loaded.size != sz) {
    g_loaded.path = path;
    g_loaded.mtime = mt;
    g_loaded.size = sz;
    g_loaded.status = load_entries(path, g_loaded.entries);
  }
  if (g_loaded.status) return g_loaded.status;
  out = g_loaded.entries;
  return KB_OK;
}

thread_local kb_tile t_last_tile{};
thread_local int t_last_cached = 0;

}  // namespace

namespace kb {

int nb_class_of(uint64_t blocks) {
  const int c = floor_log2(blocks ? blocks : 1);
  return c < KB_NB_CLASSES - 1 ? c : KB_NB_CLASSES - 1;
}

int batch_class_of(uint64_t n) { return floor_log2(n ? n : 1); }

// The tile for a batch from the file `path` (or KBATCH_TUNE when NULL).
// Returns 1 if any entry matched, 0 if none (or no file is named), <0 on a
// malformed file.
int tune_lookup_key(const char* path, const char* arch_in, const char* rocm_in, int variant,
                    uint64_t n, kb_tile* out) {
  *out = kb_tile{};
  if (!path) path = std::getenv("KBATCH_TUNE");
  if (!path || !*path) return 0;
  const char* vname = variant_name(variant);
  if (!vname) return 0;
  std::vector<Entry> es;
  int rc = entries_for(path, es);
  if (rc) return rc;
  std::string arch, rocm;
  rc = resolve_key(arch_in, rocm_in, arch, rocm);
  if (rc) return rc;
  const int bc = batch_class_of(n);
  int found = 0;
  for (const Entry& e : es) {
    if (e.arch != arch || e.rocm != rocm || e.variant != vname || e.batch_class != bc) continue;
    found = 1;
    if (e.nb_class < 0) {
      out->waves_per_simd = e.waves_per_simd;
      out->steps_per_item = e.steps_per_item;
      out->staging = e.staging;
    } else {
      out->class_steps[e.nb_class] = e.steps;
      out->class_threads[e.nb_class] = e.threads_per_state;
    }
  }
  return found;
}

int tune_lookup(const char* path, int variant, uint64_t n, kb_tile* out) {
  return tune_lookup_key(path, nullptr, nullptr, variant, n, out);
}

void note_tile(const kb_tile* t, int cached) {
  t_last_tile = t ? *t : kb_tile{};
  t_last_cached = cached;
}

}  // namespace kb

extern "C" {

int keccak_tune_store(const char* path, const char* arch_in, const char* rocm_in, int variant,
                      uint64_t n, const kb_tile* tile, double ms) {
  if (!path || !*path || !tile) return kb::set_last_error(KB_EINVAL, "NULL path or tile");
  const char* vname = variant_name(variant);
  if (!vname) return kb::set_last_error(KB_EINVAL, "variant must be -1 (mixed) or 0..3");
  if (n == 0) return kb::set_last_error(KB_EINVAL, "n must be positive");
  std::string arch, rocm;
  int rc = resolve_key(arch_in, rocm_in, arch, rocm);
  if (rc) return rc;
  std::vector<Entry> es;
  {
    std::lock_guard<std::mutex> lk(g_tmu);
    rc = load_entries(path, es);
  }
  if (rc) return rc;
  std::vector<Entry> add;
  Entry base;
  base.arch = arch;
  base.rocm = rocm;
  base.variant = vname;
  base.batch_class = kb::batch_class_of(n);
  Entry h = base;
  h.waves_per_simd = tile->waves_per_simd;
  h.steps_per_item = tile->steps_per_item;
  h.staging = tile->staging;
  h.ms = ms;
  add.push_back(h);
  for (int c = 0; c < KB_NB_CLASSES; ++c) {
    if (!tile->class_steps[c] && !tile->class_threads[c]) continue;
    Entry e = base;
    e.nb_class = c;
    e.steps = tile->class_steps[c];
    e.threads_per_state = tile->class_threads[c];
    add.push_back(e);
  }
  for (const Entry& a : add) {
    bool replaced = false;
    for (Entry& e : es)
      if (e.same_key(a)) {
        e = a;
        replaced = true;
      }
    if (!replaced) es.push_back(a);
  }
  std::lock_guard<std::mutex> lk(g_tmu);
  g_loaded.path.clear();  // force a reload on the next lookup
  return save_entries(path, es);
}

int keccak_tune_lookup(const char* path, const char* arch, const char* rocm, int variant, uint64_t n,
                       kb_tile* out) {
  if (!out) return kb::set_last_error(KB_EINVAL, "NULL output tile");
  return kb::tune_lookup_key(path, arch, rocm, variant, n, out);
}

int keccak_last_tile(kb_tile* out) {
  if (out) *out = t_last_tile;
  return t_last_cached;
}

}  // extern "C"
