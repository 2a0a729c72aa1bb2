// JSON cache of the batched plan's autotuner (host code). A small
// recursive-descent reader for the subset the writer produces (objects,
// strings, numbers; whitespace anywhere), so that a hand-edited file with the
// same shape also reads.
#include "tune_cache.hpp"

#include <cctype>
#include <cstdio>
#include <cstdlib>
#include <fstream>
#include <sstream>
#include <unistd.h>

namespace ipfb {
namespace {

struct Reader {
  const std::string& s;
  size_t i = 0;
  bool ok = true;
  explicit Reader(const std::string& t) : s(t) {}
  void ws() {
    while (i < s.size() && isspace((unsigned char)s[i])) ++i;
  }
  bool eat(char c) {
    ws();
    if (i < s.size() && s[i] == c) {
      ++i;
      return true;
    }
    return false;
  }
  bool str(std::string& out) {
    ws();
    if (i >= s.size() || s[i] != '"') return ok = false;
    ++i;
    out.clear();
    while (i < s.size() && s[i] != '"') {
      if (s[i] == '\\' && i + 1 < s.size()) ++i;
      out.push_back(s[i++]);
    }
    if (i >= s.size()) return ok = false;
    ++i;
    return true;
  }
  bool num(double& v) {
    ws();
    const char* b = s.c_str() + i;
    char* e = nullptr;
    v = strtod(b, &e);
    if (e == b) return ok = false;
    i += (size_t)(e - b);
    return true;
  }
  // skips any value (object, string, number, true/false/null)
  bool skip() {
    ws();
    if (i >= s.size()) return ok = false;
    if (s[i] == '{') {
      ++i;
      if (eat('}')) return true;
      do {
        std::string k;
        if (!str(k) || !eat(':') || !skip()) return ok = false;
      } while (eat(','));
      return eat('}') || (ok = false);
    }
    if (s[i] == '"') {
      std::string t;
      return str(t);
    }
    if (isalpha((unsigned char)s[i])) {
      while (i < s.size() && isalpha((unsigned char)s[i])) ++i;
      return true;
    }
    double v;
    return num(v);
  }
  bool entry(TuneEntry& t) {
    if (!eat('{')) return ok = false;
    if (eat('}')) return true;
    do {
      std::string k;
      if (!str(k) || !eat(':')) return ok = false;
      double v = 0.0;
      if (k == "l1" || k == "mb" || k == "kb" || k == "pchunk" || k == "fuse" || k == "nat" || k == "us") {
        if (!num(v)) return false;
        if (k == "l1") t.l1 = (int)v;
        if (k == "mb") t.mb = (int)v;
        if (k == "kb") t.kb = (int)v;
        if (k == "pchunk") t.pchunk = (int)v;
        if (k == "fuse") t.fuse = (int)v;
        if (k == "nat") t.nat = (int)v;
        if (k == "us") t.us = v;
      } else if (!skip()) {
        return false;
      }
    } while (eat(','));
    return eat('}') || (ok = false);
  }
};

bool parse(const std::string& text, std::map<std::string, TuneEntry>& out) {
  Reader r(text);
  std::map<std::string, TuneEntry> got;
  if (!r.eat('{')) return false;
  if (!r.eat('}')) {
    do {
      std::string k;
      if (!r.str(k) || !r.eat(':')) return false;
      if (k == "entries") {
        if (!r.eat('{')) return false;
        if (!r.eat('}')) {
          do {
            std::string key;
            TuneEntry t;
            if (!r.str(key) || !r.eat(':') || !r.entry(t)) return false;
            got[key] = t;
          } while (r.eat(','));
          if (!r.eat('}')) return false;
        }
      } else if (!r.skip()) {
        return false;
      }
    } while (r.eat(','));
    if (!r.eat('}')) return false;
  }
  r.ws();
  if (r.i != text.size() || !r.ok) return false;
  for (auto& kv : got) out[kv.first] = kv.second;
  return true;
}

}  // namespace

bool tune_cache_read(const std::string& path, std::map<std::string, TuneEntry>& out) {
  std::ifstream f(path);
  if (!f) return true;  // no cache yet
  std::stringstream ss;
  ss << f.rdbuf();
  return parse(ss.str(), out);
}

bool tune_cache_write(const std::string& path, const std::map<std::string, TuneEntry>& entries) {
  std::map<std::string, TuneEntry> all;
  tune_cache_read(path, all);  // an unreadable file is replaced
  for (auto& kv : entries) all[kv.first] = kv.second;
  const std::string tmp = path + ".tmp." + std::to_string((long)getpid());
  {
    std::ofstream f(tmp);
    if (!f) return false;
    f << "{\"version\": 1, \"entries\": {";
    bool first = true;
    for (auto& kv : all) {
      std::string k;
      for (char c : kv.first) {
        if (c == '"' || c == '\\') k.push_back('\\');
        k.push_back(c);
      }
      char buf[160];
      snprintf(buf, sizeof(buf),
               "{\"l1\": %d, \"mb\": %d, \"kb\": %d, \"pchunk\": %d, \"fuse\": %d, \"nat\": %d, \"us\": %.3f}",
               kv.second.l1, kv.second.mb, kv.second.kb, kv.second.pchunk, kv.second.fuse, kv.second.nat, kv.second.us);
      f << (first ? "\n  \"" : ",\n  \"") << k << "\": " << buf;
      first = false;
    }
    f << "\n}}\n";
    if (!f) return false;
  }
  if (rename(tmp.c_str(), path.c_str()) != 0) {
    remove(tmp.c_str());
    return false;
  }
  return true;
}

}  // namespace ipfb
