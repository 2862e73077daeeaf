// Cache of the autotuner's measured choices (host only): keys, nearest-size lookup
// and the JSON file format. None of these choices changes a result bit; they only
// select among launch shapes of the same arithmetic.
//
// Keys name the parameters a choice was measured for:
//   product  "N<N>.P<P>.K<K>.M<M>.n<n_o>.r<raw>.T<bucket>"
//   batch    "N<N>.P<P>.batch<n>.r<raw>.T<bucket>"
// with the token count rounded up to a power of two (bucket). The file:
//   {"device": "<arch|name|compute units>",
//    "entries": [{"key": "...", "method": 1, "tt_log2": 3, "order": 0, "launch": 0,
//                 "ms": 9.1}, ...]}
// Entries recorded for another device are not loaded.
#pragma once

#include <stdint.h>
#include <stdio.h>
#include <stdlib.h>

#include <map>
#include <string>
#include <vector>

#include "rlwe.h"

namespace rlwe {
namespace tune {

inline uint32_t tbucket(uint32_t T) {
  uint32_t b = 1;
  while (b < T && b < (1u << 30)) b <<= 1;
  return b;
}

inline std::string product_key(uint32_t N, uint32_t P, uint32_t K, uint32_t M, uint32_t n_o,
                               uint32_t raw, uint32_t T) {
  char buf[160];
  snprintf(buf, sizeof buf, "N%u.P%u.K%u.M%u.n%u.r%u.T%u", N, P, K, M, n_o, raw ? 1u : 0u,
           tbucket(T));
  return buf;
}

inline std::string batch_key(uint32_t N, uint32_t P, uint32_t n, uint32_t raw, uint32_t T) {
  char buf[160];
  snprintf(buf, sizeof buf, "N%u.P%u.batch%u.r%u.T%u", N, P, n, raw ? 1u : 0u, tbucket(T));
  return buf;
}

// Fields of a product key (kind 0) or batch key (kind 1), for nearest-size lookups.
struct KeyFields {
  int kind = -1;
  uint32_t N = 0, P = 0, K = 0, M = 0, n_o = 0, n = 0, raw = 0, T = 0;
};
inline KeyFields parse_key(const std::string& k) {
  KeyFields f;
  if (sscanf(k.c_str(), "N%u.P%u.K%u.M%u.n%u.r%u.T%u", &f.N, &f.P, &f.K, &f.M, &f.n_o, &f.raw,
             &f.T) == 7)
    f.kind = 0;
  else if (sscanf(k.c_str(), "N%u.P%u.batch%u.r%u.T%u", &f.N, &f.P, &f.n, &f.raw, &f.T) == 5)
    f.kind = 1;
  return f;
}

struct Cache {
  std::string device;
  std::map<std::string, rlwe_schedule> entries;
};

inline int log2_distance(uint32_t a, uint32_t b) {
  int d = 0;
  while (a < b) {
    a <<= 1;
    ++d;
  }
  while (b < a) {
    b <<= 1;
    ++d;
  }
  return d;
}

// The entry of this product shape at the token bucket of T, else at the nearest bucket
// (ties: the larger one).
inline bool find_product(const Cache& c, uint32_t N, uint32_t P, uint32_t K, uint32_t M,
                         uint32_t n_o, uint32_t raw, uint32_t T, rlwe_schedule* out) {
  const uint32_t b = tbucket(T);
  int best = 1 << 30;
  uint32_t bestT = 0;
  for (const auto& e : c.entries) {
    const KeyFields f = parse_key(e.first);
    if (f.kind != 0 || f.N != N || f.P != P || f.K != K || f.M != M || f.n_o != n_o ||
        f.raw != (raw ? 1u : 0u))
      continue;
    const int d = log2_distance(f.T, b);
    if (d < best || (d == best && f.T > bestT)) {
      best = d;
      bestT = f.T;
      *out = e.second;
    }
  }
  return bestT != 0;
}

// Method for loading an orientation (K inputs, M outputs, one row per polynomial): the
// switched-output entry with the largest token bucket of that shape.
inline bool find_method(const Cache& c, uint32_t N, uint32_t P, uint32_t K, uint32_t M,
                        uint32_t* method) {
  uint32_t bestT = 0;
  for (const auto& e : c.entries) {
    const KeyFields f = parse_key(e.first);
    if (f.kind == 0 && f.N == N && f.P == P && f.K == K && f.M == M && f.n_o == 1 && f.raw == 0 &&
        f.T > bestT) {
      bestT = f.T;
      *method = e.second.method;
    }
  }
  return bestT != 0;
}

// The batch entry of n products at the bucket of their largest token count, else at the
// nearest bucket for n products.
inline bool find_batch(const Cache& c, uint32_t N, uint32_t P, uint32_t n, uint32_t raw,
                       uint32_t T, rlwe_schedule* out) {
  const uint32_t b = tbucket(T);
  int best = 1 << 30;
  uint32_t bestT = 0;
  for (const auto& e : c.entries) {
    const KeyFields f = parse_key(e.first);
    if (f.kind != 1 || f.N != N || f.P != P || f.n != n || f.raw != (raw ? 1u : 0u)) continue;
    const int d = log2_distance(f.T, b);
    if (d < best || (d == best && f.T > bestT)) {
      best = d;
      bestT = f.T;
      *out = e.second;
    }
  }
  return bestT != 0;
}

inline std::string json_escape(const std::string& s) {
  std::string o;
  for (char ch : s) {
    if (ch == '"' || ch == '\\') o += '\\';
    if ((unsigned char)ch >= 0x20) o += ch;
  }
  return o;
}

inline std::string to_json(const Cache& c) {
  std::string o = "{\"device\": \"" + json_escape(c.device) + "\",\n \"entries\": [";
  bool first = true;
  for (const auto& e : c.entries) {
    char buf[320];
    snprintf(buf, sizeof buf,
             "%s\n  {\"key\": \"%s\", \"method\": %u, \"tt_log2\": %u, \"order\": %u, "
             "\"launch\": %u, \"ms\": %.6g}",
             first ? "" : ",", json_escape(e.first).c_str(), e.second.method, e.second.tt_log2,
             e.second.order, e.second.launch, (double)e.second.ms);
    o += buf;
    first = false;
  }
  o += "\n]}\n";
  return o;
}

// A small JSON reader for the file above: objects, arrays, strings (escapes \" and \\),
// numbers, true, false, null.
struct JVal {
  enum Kind { NUL, NUM, STR, ARR, OBJ, BOOL } kind = NUL;
  double num = 0;
  std::string str;
  std::vector<JVal> arr;
  std::vector<std::pair<std::string, JVal>> obj;
  const JVal* get(const char* k) const {
    for (const auto& kv : obj)
      if (kv.first == k) return &kv.second;
    return nullptr;
  }
};

struct JParser {
  const std::string& s;
  size_t i = 0;
  std::string err;
  explicit JParser(const std::string& text) : s(text) {}
  void ws() {
    while (i < s.size() && (s[i] == ' ' || s[i] == '\n' || s[i] == '\r' || s[i] == '\t')) ++i;
  }
  bool fail(const char* what) {
    if (err.empty()) {
      char buf[96];
      snprintf(buf, sizeof buf, "%s at byte %zu", what, i);
      err = buf;
    }
    return false;
  }
  bool string(std::string* out) {
    if (i >= s.size() || s[i] != '"') return fail("expected a string");
    ++i;
    out->clear();
    while (i < s.size() && s[i] != '"') {
      if (s[i] == '\\') {
        if (++i >= s.size()) return fail("unterminated escape");
        if (s[i] != '"' && s[i] != '\\') return fail("unsupported escape");
      }
      *out += s[i++];
    }
    if (i >= s.size()) return fail("unterminated string");
    ++i;
    return true;
  }
  bool value(JVal* v, int depth) {
    if (depth > 16) return fail("nested too deeply");
    ws();
    if (i >= s.size()) return fail("unexpected end");
    const char ch = s[i];
    if (ch == '{') {
      v->kind = JVal::OBJ;
      ++i;
      ws();
      if (i < s.size() && s[i] == '}') return ++i, true;
      for (;;) {
        ws();
        std::string k;
        if (!string(&k)) return false;
        ws();
        if (i >= s.size() || s[i] != ':') return fail("expected ':'");
        ++i;
        JVal x;
        if (!value(&x, depth + 1)) return false;
        v->obj.emplace_back(k, x);
        ws();
        if (i < s.size() && s[i] == ',') {
          ++i;
          continue;
        }
        if (i < s.size() && s[i] == '}') return ++i, true;
        return fail("expected ',' or '}'");
      }
    }
    if (ch == '[') {
      v->kind = JVal::ARR;
      ++i;
      ws();
      if (i < s.size() && s[i] == ']') return ++i, true;
      for (;;) {
        JVal x;
        if (!value(&x, depth + 1)) return false;
        v->arr.push_back(x);
        ws();
        if (i < s.size() && s[i] == ',') {
          ++i;
          continue;
        }
        if (i < s.size() && s[i] == ']') return ++i, true;
        return fail("expected ',' or ']'");
      }
    }
    if (ch == '"') {
      v->kind = JVal::STR;
      return string(&v->str);
    }
    if (s.compare(i, 4, "true") == 0 || s.compare(i, 5, "false") == 0) {
      v->kind = JVal::BOOL;
      v->num = s[i] == 't' ? 1 : 0;
      i += s[i] == 't' ? 4 : 5;
      return true;
    }
    if (s.compare(i, 4, "null") == 0) {
      i += 4;
      return true;
    }
    char* end = nullptr;
    const double d = strtod(s.c_str() + i, &end);
    if (end == s.c_str() + i) return fail("unexpected character");
    v->kind = JVal::NUM;
    v->num = d;
    i = (size_t)(end - s.c_str());
    return true;
  }
};

// Adds the file's entries to c when they were recorded for c's device; *loaded = their
// number (0 for another device). Returns false with *err on a malformed file.
inline bool from_json(const std::string& text, Cache* c, size_t* loaded, std::string* err) {
  *loaded = 0;
  JParser p(text);
  JVal root;
  if (!p.value(&root, 0)) {
    *err = p.err;
    return false;
  }
  const JVal* dev = root.get("device");
  const JVal* ent = root.get("entries");
  if (root.kind != JVal::OBJ || !dev || dev->kind != JVal::STR || !ent || ent->kind != JVal::ARR) {
    *err = "expected {\"device\": ..., \"entries\": [...]}";
    return false;
  }
  std::map<std::string, rlwe_schedule> got;
  for (const JVal& e : ent->arr) {
    const JVal* k = e.get("key");
    const char* names[] = {"method", "tt_log2", "order", "launch", "ms"};
    const JVal* f[5];
    bool okk = e.kind == JVal::OBJ && k && k->kind == JVal::STR && parse_key(k->str).kind >= 0;
    for (int x = 0; x < 5 && okk; ++x) {
      f[x] = e.get(names[x]);
      okk = f[x] && f[x]->kind == JVal::NUM;
    }
    if (!okk) {
      *err = "malformed entry";
      return false;
    }
    rlwe_schedule sc{};
    sc.method = (uint32_t)f[0]->num;
    sc.tt_log2 = (uint32_t)f[1]->num;
    sc.order = (uint32_t)f[2]->num;
    sc.launch = (uint32_t)f[3]->num;
    sc.ms = (float)f[4]->num;
    if (sc.method > 1 || sc.tt_log2 > 5 || sc.order > 1 || sc.launch > 1) {
      *err = "entry out of range: " + k->str;
      return false;
    }
    got[k->str] = sc;
  }
  if (dev->str != c->device) return true;
  for (const auto& kv : got) c->entries[kv.first] = kv.second;
  *loaded = got.size();
  return true;
}

}  // namespace tune
}  // namespace rlwe

struct rlwe_tuner {
  rlwe::tune::Cache cache;
};
