// Autotuner state: measured FFT-pair costs per single-pass length and the
// schedules the uneven batch picked, kept per device architecture and
// persisted as JSON so that a later process starts from them.
//
// File (path from TZ_TUNE_CACHE; else $XDG_CACHE_HOME/thzspec/tune.json or
// $HOME/.cache/thzspec/tune.json; "off" or "" disables reading and writing):
//   {"format": 1, "entries": {"<arch>/<library version>": {
//       "fft_pair_ns": {"256": t, ..., "16384": t},
//       "batches": {"<job-table hash>": {"topology": i, "inner": i, "ms": t}}}}}
// An entry is used only under the exact key of the current device and
// library; a file that does not parse is ignored as a whole (defaults) and
// replaced at the next write.
#include <hip/hip_runtime.h>
#include <math.h>
#include <stdio.h>
#include <stdlib.h>
#include <string.h>
#include <sys/stat.h>
#include <unistd.h>

#include <algorithm>
#include <map>
#include <memory>
#include <mutex>
#include <string>
#include <utility>
#include <vector>

#include "internal.h"
#include "thzspec.h"

namespace tz {

namespace {

// ---------------------------------------------------------------------------
// a small JSON value: objects, arrays, strings, numbers (all the file holds)
// ---------------------------------------------------------------------------
struct JVal {
  enum Kind { Null, Num, Str, Obj, Arr } kind = Null;
  double num = 0.0;
  std::string str;
  std::vector<std::pair<std::string, JVal>> obj;
  std::vector<JVal> arr;
  const JVal *get(const std::string &k) const {
    if (kind != Obj) return nullptr;
    for (auto &kv : obj)
      if (kv.first == k) return &kv.second;
    return nullptr;
  }
  JVal &set(const std::string &k) {
    kind = Obj;
    for (auto &kv : obj)
      if (kv.first == k) return kv.second;
    obj.emplace_back(k, JVal());
    return obj.back().second;
  }
};

struct Parser {
  const char *p, *end;
  std::string err;
  void ws() {
    while (p < end && (*p == ' ' || *p == '\n' || *p == '\r' || *p == '\t')) ++p;
  }
  bool fail(const char *what) {
    if (err.empty()) err = what;
    return false;
  }
  bool string(std::string *out) {
    if (p >= end || *p != '"') return fail("expected a string");
    ++p;
    out->clear();
    while (p < end && *p != '"') {
      if (*p == '\\') {
        if (++p >= end) return fail("unterminated escape");
        const char c = *p;
        if (c == '"' || c == '\\' || c == '/')
          out->push_back(c);
        else if (c == 'n')
          out->push_back('\n');
        else if (c == 't')
          out->push_back('\t');
        else
          return fail("unsupported escape");
        ++p;
      } else {
        out->push_back(*p++);
      }
    }
    if (p >= end) return fail("unterminated string");
    ++p;
    return true;
  }
  bool value(JVal *v, int depth) {
    if (depth > 16) return fail("nested too deeply");
    ws();
    if (p >= end) return fail("unexpected end");
    if (*p == '{') {
      ++p;
      v->kind = JVal::Obj;
      ws();
      if (p < end && *p == '}') return ++p, true;
      for (;;) {
        ws();
        std::string k;
        if (!string(&k)) return false;
        ws();
        if (p >= end || *p != ':') return fail("expected ':'");
        ++p;
        JVal c;
        if (!value(&c, depth + 1)) return false;
        v->obj.emplace_back(std::move(k), std::move(c));
        ws();
        if (p < end && *p == ',') {
          ++p;
          continue;
        }
        if (p < end && *p == '}') return ++p, true;
        return fail("expected ',' or '}'");
      }
    }
    if (*p == '[') {
      ++p;
      v->kind = JVal::Arr;
      ws();
      if (p < end && *p == ']') return ++p, true;
      for (;;) {
        JVal c;
        if (!value(&c, depth + 1)) return false;
        v->arr.push_back(std::move(c));
        ws();
        if (p < end && *p == ',') {
          ++p;
          continue;
        }
        if (p < end && *p == ']') return ++p, true;
        return fail("expected ',' or ']'");
      }
    }
    if (*p == '"') {
      v->kind = JVal::Str;
      return string(&v->str);
    }
    if (end - p >= 4 && !strncmp(p, "null", 4)) {
      p += 4;
      v->kind = JVal::Null;
      return true;
    }
    char *q = nullptr;
    const std::string tok(p, (size_t)std::min<ptrdiff_t>(end - p, 64));
    const double d = strtod(tok.c_str(), &q);
    if (q == tok.c_str()) return fail("unexpected character");
    p += q - tok.c_str();
    v->kind = JVal::Num;
    v->num = d;
    return true;
  }
};

bool parse_json(const std::string &text, JVal *out, std::string *err) {
  Parser ps{text.data(), text.data() + text.size(), {}};
  if (!ps.value(out, 0)) {
    *err = ps.err;
    return false;
  }
  ps.ws();
  if (ps.p != ps.end) {
    *err = "trailing characters";
    return false;
  }
  return true;
}

void dump(const JVal &v, std::string *o, int ind) {
  const std::string pad(ind + 1, ' ');
  switch (v.kind) {
    case JVal::Null: *o += "null"; break;
    case JVal::Num: {
      char b[40];
      snprintf(b, sizeof b, "%.9g", v.num);
      *o += b;
      break;
    }
    case JVal::Str: *o += "\"" + v.str + "\""; break;  // keys and names hold no quotes or escapes
    case JVal::Arr:
      *o += "[";
      for (size_t i = 0; i < v.arr.size(); ++i) {
        if (i) *o += ", ";
        dump(v.arr[i], o, ind);
      }
      *o += "]";
      break;
    case JVal::Obj:
      *o += "{\n";
      for (size_t i = 0; i < v.obj.size(); ++i) {
        *o += pad + "\"" + v.obj[i].first + "\": ";
        dump(v.obj[i].second, o, ind + 1);
        *o += i + 1 < v.obj.size() ? ",\n" : "\n";
      }
      *o += std::string(ind, ' ') + "}";
      break;
  }
}

// ---------------------------------------------------------------------------
// process state
// ---------------------------------------------------------------------------
struct ArchTune {
  bool have_pair = false;
  double pair_ns[15] = {};  // per log2 L, time of one FFT pair (ns)
  std::map<std::string, BatchTune> batches;
};

struct TuneState {
  std::mutex mu;
  bool loaded = false;
  std::string path;    // resolved cache path ("" = persistence off)
  std::string status;  // outcome of the last load or save
  JVal file;           // the whole parsed file (kept so other keys survive a save)
  std::map<std::string, ArchTune> arch;  // by "<arch>/<version>"
  std::string cur_key;                   // key of the current device ("" = none)
};

TuneState &state() {
  static TuneState *s = new TuneState();  // lives until the process ends
  return *s;
}

std::string resolve_path() {
  const char *e = getenv("TZ_TUNE_CACHE");
  if (e) return (!*e || !strcmp(e, "off")) ? std::string() : std::string(e);
  if (const char *x = getenv("XDG_CACHE_HOME"); x && *x) return std::string(x) + "/thzspec/tune.json";
  if (const char *h = getenv("HOME"); h && *h) return std::string(h) + "/.cache/thzspec/tune.json";
  return std::string();
}

std::string device_key() {
  int dev = 0, n = 0;
  if (hipGetDeviceCount(&n) != hipSuccess || n < 1) {
    (void)hipGetLastError();
    return std::string();
  }
  if (hipGetDevice(&dev) != hipSuccess) return std::string();
  hipDeviceProp_t prop;
  if (hipGetDeviceProperties(&prop, dev) != hipSuccess) return std::string();
  return std::string(prop.gcnArchName) + "/" + tz_version();
}

void absorb(const JVal &root, TuneState &s) {
  const JVal *ents = root.get("entries");
  if (!ents || ents->kind != JVal::Obj) return;
  for (auto &kv : ents->obj) {
    ArchTune t;
    if (const JVal *f = kv.second.get("fft_pair_ns")) {
      int got = 0;
      for (int c = 8; c <= 14; ++c) {
        const JVal *v = f->get(std::to_string(1 << c));
        if (v && v->kind == JVal::Num && v->num > 0.0 && isfinite(v->num)) {
          t.pair_ns[c] = v->num;
          ++got;
        }
      }
      t.have_pair = got == 7;  // all seven lengths or none
    }
    if (const JVal *bs = kv.second.get("batches"); bs && bs->kind == JVal::Obj)
      for (auto &b : bs->obj) {
        const JVal *tp = b.second.get("topology"), *in = b.second.get("inner"), *ms = b.second.get("ms");
        if (!tp || !in || tp->kind != JVal::Num || in->kind != JVal::Num) continue;
        BatchTune bt;
        bt.topology = (int)tp->num;
        bt.inner = (int)in->num;
        bt.ms = ms && ms->kind == JVal::Num ? ms->num : -1.0;
        if (bt.topology < 0 || bt.topology > 3 || bt.inner < 0 || bt.inner > 1) continue;
        t.batches[b.first] = bt;
      }
    s.arch[kv.first] = t;
  }
}

// (re)load when first used or when TZ_TUNE_CACHE names another file
void ensure_loaded(TuneState &s) {
  const std::string path = resolve_path();
  if (s.loaded && path == s.path) return;
  s.loaded = true;
  s.path = path;
  s.arch.clear();
  s.file = JVal();
  s.cur_key = device_key();
  if (path.empty()) {
    s.status = "persistence off";
    return;
  }
  FILE *f = fopen(path.c_str(), "rb");
  if (!f) {
    s.status = "no cache file";
    return;
  }
  std::string text;
  char buf[4096];
  size_t n;
  while ((n = fread(buf, 1, sizeof buf, f)) > 0 && text.size() < ((size_t)16 << 20)) text.append(buf, n);
  fclose(f);
  JVal root;
  std::string err;
  if (!parse_json(text, &root, &err) || root.kind != JVal::Obj || !root.get("format") ||
      root.get("format")->kind != JVal::Num || root.get("format")->num != 1.0) {
    s.status = "cache ignored (" + (err.empty() ? std::string("not a format-1 tune file") : err) + ")";
    tz_log("autotune: %s: %s", path.c_str(), s.status.c_str());
    return;
  }
  s.file = root;
  absorb(root, s);
  s.status = s.cur_key.empty() ? "cache read, no device"
             : s.arch.count(s.cur_key) ? "cache entry for " + s.cur_key
                                       : "cache has no entry for " + s.cur_key;
  tz_log("autotune: %s: %s", path.c_str(), s.status.c_str());
}

// write the current device's entry into the file (atomically: temp + rename)
void save(TuneState &s) {
  if (s.path.empty() || s.cur_key.empty()) return;
  const ArchTune &t = s.arch[s.cur_key];
  JVal root = s.file.kind == JVal::Obj ? s.file : JVal();
  root.set("format").kind = JVal::Num;
  root.set("format").num = 1.0;
  JVal &ent = root.set("entries").set(s.cur_key);
  ent.kind = JVal::Obj;
  if (t.have_pair) {
    JVal &f = ent.set("fft_pair_ns");
    for (int c = 8; c <= 14; ++c) {
      JVal &v = f.set(std::to_string(1 << c));
      v.kind = JVal::Num;
      v.num = t.pair_ns[c];
    }
  }
  JVal &bs = ent.set("batches");
  bs.kind = JVal::Obj;
  for (auto &b : t.batches) {
    JVal &e = bs.set(b.first);
    e.set("topology").kind = JVal::Num;
    e.set("topology").num = b.second.topology;
    e.set("inner").kind = JVal::Num;
    e.set("inner").num = b.second.inner;
    e.set("ms").kind = JVal::Num;
    e.set("ms").num = b.second.ms;
  }
  s.file = root;
  std::string text;
  dump(root, &text, 0);
  text += "\n";
  // parent directories (best effort)
  for (size_t i = 1; i < s.path.size(); ++i)
    if (s.path[i] == '/') (void)mkdir(s.path.substr(0, i).c_str(), 0755);
  const std::string tmp = s.path + ".tmp." + std::to_string((long long)getpid());
  FILE *f = fopen(tmp.c_str(), "wb");
  bool ok = f && fwrite(text.data(), 1, text.size(), f) == text.size();
  if (f) ok = (fclose(f) == 0) && ok;
  if (ok) ok = rename(tmp.c_str(), s.path.c_str()) == 0;
  if (!ok) {
    (void)remove(tmp.c_str());
    s.status = "cache not written (" + s.path + ")";
  } else {
    s.status = "cache entry for " + s.cur_key + " written";
  }
  tz_log("autotune: %s", s.status.c_str());
}

}  // namespace

// Relative time of one workgroup FFT pair of length L.  Measured per device
// by tz_autotune (or read from the cache); otherwise the built-in table:
// about the same per point up to 4096, about 1.35x per point at 8192 and
// 2.1x at 16384 (the register and LDS pressure of the longest transforms).
double fft_pair_cost(int64_t L) {
  TuneState &s = state();
  {
    std::lock_guard<std::mutex> g(s.mu);
    ensure_loaded(s);
    auto it = s.arch.find(s.cur_key);
    if (!s.cur_key.empty() && it != s.arch.end() && it->second.have_pair) {
      int c = 0;
      while ((1LL << c) < L) ++c;
      if (c >= 8 && c <= 14) return it->second.pair_ns[c];
    }
  }
  return (double)L * (L <= 4096 ? 1.0 : (L <= 8192 ? 1.35 : 2.1));
}

bool tune_batch_lookup(const std::string &sig, BatchTune *out) {
  TuneState &s = state();
  std::lock_guard<std::mutex> g(s.mu);
  ensure_loaded(s);
  auto it = s.arch.find(s.cur_key);
  if (s.cur_key.empty() || it == s.arch.end()) return false;
  auto b = it->second.batches.find(sig);
  if (b == it->second.batches.end()) return false;
  *out = b->second;
  return true;
}

void tune_batch_store(const std::string &sig, const BatchTune &t) {
  TuneState &s = state();
  std::lock_guard<std::mutex> g(s.mu);
  ensure_loaded(s);
  if (s.cur_key.empty()) return;
  s.arch[s.cur_key].batches[sig] = t;
  save(s);
}

void tune_set_pair_costs(const double ns[15]) {
  TuneState &s = state();
  std::lock_guard<std::mutex> g(s.mu);
  ensure_loaded(s);
  if (s.cur_key.empty()) return;
  ArchTune &t = s.arch[s.cur_key];
  for (int c = 8; c <= 14; ++c) t.pair_ns[c] = ns[c];
  t.have_pair = true;
  save(s);
}

}  // namespace tz

extern "C" int64_t tz_tune_describe(char *buf, int64_t len) {
  using namespace tz;
  TuneState &s = state();
  std::string d;
  {
    std::lock_guard<std::mutex> g(s.mu);
    ensure_loaded(s);
    d = "cache=" + (s.path.empty() ? std::string("off") : s.path) + "; status=" + s.status +
        "; device=" + (s.cur_key.empty() ? std::string("none") : s.cur_key);
    auto it = s.arch.find(s.cur_key);
    const bool have = !s.cur_key.empty() && it != s.arch.end();
    if (have && it->second.have_pair) {
      d += "; fft_pair_ns=measured:";
      for (int c = 8; c <= 14; ++c) {
        char t[40];
        snprintf(t, sizeof t, " %d=%.1f", 1 << c, it->second.pair_ns[c]);
        d += t;
      }
    } else {
      d += "; fft_pair_ns=built-in";
    }
    d += "; batches=" + std::to_string(have ? it->second.batches.size() : 0);
  }
  if (buf && len > 0) {
    const size_t n = std::min<size_t>((size_t)len - 1, d.size());
    memcpy(buf, d.data(), n);
    buf[n] = 0;
  }
  return (int64_t)d.size();
}
