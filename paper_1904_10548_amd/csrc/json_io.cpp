// JSON front-end (Sec. 5.1, Table of classes and their JSON files): the
// network, the scenario tree, the forecaster, the controller configuration,
// the plant state and the control output, read and written as JSON files.
// The paper names the files but not their fields; the formats here are this
// library's own and are spelled out in tapg.h.  Reading is strict: unknown
// keys, wrong shapes and non-finite numbers are errors naming the file, the
// key and (for syntax errors) the line and column.
//
// Every reader parses into plain arrays and then calls the array entry points
// (tapg_network_create, tapg_tree_create, ...), so a model read from JSON is
// validated exactly like one passed as arrays.
#include <charconv>
#include <cmath>
#include <cstdio>
#include <cstring>
#include <fstream>
#include <initializer_list>
#include <sstream>
#include <string>
#include <utility>
#include <vector>

#include "internal.h"

using namespace tapg;

namespace {

// ---------------------------------------------------------------- values --

struct JVal {
  enum Kind { Null, Bool, Num, Str, Arr, Obj } kind = Null;
  bool b = false;
  double num = 0.0;
  std::string str;
  std::vector<JVal> arr;
  std::vector<std::pair<std::string, JVal>> obj;
};

const char* kind_name(JVal::Kind k) {
  switch (k) {
    case JVal::Null: return "null";
    case JVal::Bool: return "a boolean";
    case JVal::Num: return "a number";
    case JVal::Str: return "a string";
    case JVal::Arr: return "an array";
    default: return "an object";
  }
}

// ---------------------------------------------------------------- parser --

class Parser {
 public:
  Parser(const std::string& text, const std::string& file) : s_(text), file_(file) {}

  JVal document() {
    JVal v = value(0);
    ws();
    if (i_ != s_.size()) error("unexpected text after the top-level value");
    return v;
  }

 private:
  static constexpr int kMaxDepth = 64;
  const std::string& s_;
  const std::string& file_;
  size_t i_ = 0;

  [[noreturn]] void error(const std::string& what) const {
    int line = 1, col = 1;
    for (size_t k = 0; k < i_ && k < s_.size(); ++k) {
      if (s_[k] == '\n') {
        ++line;
        col = 1;
      } else {
        ++col;
      }
    }
    throw Fail{TAPG_EINVAL, file_ + ":" + std::to_string(line) + ":" + std::to_string(col) +
                                ": " + what};
  }

  void ws() {
    while (i_ < s_.size() && (s_[i_] == ' ' || s_[i_] == '\t' || s_[i_] == '\n' || s_[i_] == '\r'))
      ++i_;
  }

  bool literal(const char* word) {
    const size_t n = std::strlen(word);
    if (s_.compare(i_, n, word) != 0) return false;
    i_ += n;
    return true;
  }

  JVal value(int depth) {
    if (depth > kMaxDepth) error("nesting deeper than 64 levels");
    ws();
    if (i_ >= s_.size()) error("unexpected end of file");
    JVal v;
    const char c = s_[i_];
    if (c == '{') {
      v.kind = JVal::Obj;
      ++i_;
      ws();
      if (i_ < s_.size() && s_[i_] == '}') {
        ++i_;
        return v;
      }
      for (;;) {
        ws();
        if (i_ >= s_.size() || s_[i_] != '"') error("expected a key string");
        std::string key = string();
        for (const auto& kv : v.obj)
          if (kv.first == key) error("duplicate key \"" + key + "\"");
        ws();
        if (i_ >= s_.size() || s_[i_] != ':') error("expected ':'");
        ++i_;
        v.obj.emplace_back(std::move(key), value(depth + 1));
        ws();
        if (i_ < s_.size() && s_[i_] == ',') {
          ++i_;
          continue;
        }
        if (i_ < s_.size() && s_[i_] == '}') {
          ++i_;
          return v;
        }
        error("expected ',' or '}'");
      }
    }
    if (c == '[') {
      v.kind = JVal::Arr;
      ++i_;
      ws();
      if (i_ < s_.size() && s_[i_] == ']') {
        ++i_;
        return v;
      }
      for (;;) {
        v.arr.push_back(value(depth + 1));
        ws();
        if (i_ < s_.size() && s_[i_] == ',') {
          ++i_;
          continue;
        }
        if (i_ < s_.size() && s_[i_] == ']') {
          ++i_;
          return v;
        }
        error("expected ',' or ']'");
      }
    }
    if (c == '"') {
      v.kind = JVal::Str;
      v.str = string();
      return v;
    }
    if (literal("true")) {
      v.kind = JVal::Bool;
      v.b = true;
      return v;
    }
    if (literal("false")) {
      v.kind = JVal::Bool;
      return v;
    }
    if (literal("null")) return v;
    if (c == '-' || (c >= '0' && c <= '9')) {
      v.kind = JVal::Num;
      v.num = number();
      return v;
    }
    error(std::string("unexpected character '") + c + "'");
  }

  // RFC 8259 number grammar, converted with from_chars (correctly rounded,
  // independent of the C locale).
  double number() {
    const size_t b = i_;
    auto digits = [&] {
      const size_t d0 = i_;
      while (i_ < s_.size() && s_[i_] >= '0' && s_[i_] <= '9') ++i_;
      return i_ - d0;
    };
    if (s_[i_] == '-') ++i_;
    if (i_ < s_.size() && s_[i_] == '0') {
      ++i_;
    } else if (digits() == 0) {
      error("malformed number");
    }
    if (i_ < s_.size() && s_[i_] == '.') {
      ++i_;
      if (digits() == 0) error("malformed number: digits expected after '.'");
    }
    if (i_ < s_.size() && (s_[i_] == 'e' || s_[i_] == 'E')) {
      ++i_;
      if (i_ < s_.size() && (s_[i_] == '+' || s_[i_] == '-')) ++i_;
      if (digits() == 0) error("malformed number: digits expected in the exponent");
    }
    double x = 0.0;
    const char* first = s_.data() + b;
    const char* last = s_.data() + i_;
    const auto r = std::from_chars(first, last, x);  // takes the leading '-' itself
    if (r.ec != std::errc() || r.ptr != last) error("number out of range");
    return x;
  }

  static void utf8(std::string& out, unsigned cp) {
    if (cp < 0x80) {
      out += (char)cp;
    } else if (cp < 0x800) {
      out += (char)(0xC0 | (cp >> 6));
      out += (char)(0x80 | (cp & 0x3F));
    } else if (cp < 0x10000) {
      out += (char)(0xE0 | (cp >> 12));
      out += (char)(0x80 | ((cp >> 6) & 0x3F));
      out += (char)(0x80 | (cp & 0x3F));
    } else {
      out += (char)(0xF0 | (cp >> 18));
      out += (char)(0x80 | ((cp >> 12) & 0x3F));
      out += (char)(0x80 | ((cp >> 6) & 0x3F));
      out += (char)(0x80 | (cp & 0x3F));
    }
  }

  unsigned hex4() {
    if (i_ + 4 > s_.size()) error("truncated \\u escape");
    unsigned v = 0;
    for (int k = 0; k < 4; ++k) {
      const char h = s_[i_++];
      v <<= 4;
      if (h >= '0' && h <= '9') v |= (unsigned)(h - '0');
      else if (h >= 'a' && h <= 'f') v |= (unsigned)(h - 'a' + 10);
      else if (h >= 'A' && h <= 'F') v |= (unsigned)(h - 'A' + 10);
      else error("bad hex digit in \\u escape");
    }
    return v;
  }

  std::string string() {
    ++i_;  // opening quote
    std::string out;
    for (;;) {
      if (i_ >= s_.size()) error("unterminated string");
      const unsigned char c = (unsigned char)s_[i_++];
      if (c == '"') return out;
      if (c < 0x20) error("control character in a string");
      if (c != '\\') {
        out += (char)c;
        continue;
      }
      if (i_ >= s_.size()) error("unterminated string");
      const char e = s_[i_++];
      switch (e) {
        case '"': out += '"'; break;
        case '\\': out += '\\'; break;
        case '/': out += '/'; break;
        case 'b': out += '\b'; break;
        case 'f': out += '\f'; break;
        case 'n': out += '\n'; break;
        case 'r': out += '\r'; break;
        case 't': out += '\t'; break;
        case 'u': {
          unsigned cp = hex4();
          if (cp >= 0xD800 && cp < 0xDC00) {
            if (!(i_ + 1 < s_.size() && s_[i_] == '\\' && s_[i_ + 1] == 'u'))
              error("unpaired surrogate in \\u escape");
            i_ += 2;
            const unsigned lo = hex4();
            if (lo < 0xDC00 || lo >= 0xE000) error("unpaired surrogate in \\u escape");
            cp = 0x10000 + ((cp - 0xD800) << 10) + (lo - 0xDC00);
          } else if (cp >= 0xDC00 && cp < 0xE000) {
            error("unpaired surrogate in \\u escape");
          }
          utf8(out, cp);
          break;
        }
        default: error(std::string("bad escape '\\") + e + "'");
      }
    }
  }
};

JVal read_json(const char* path, const char* what) {
  if (!path) throw Fail{TAPG_EINVAL, std::string(what) + ": NULL path"};
  std::ifstream f(path, std::ios::binary);
  if (!f) throw Fail{TAPG_EINVAL, std::string(what) + ": cannot open " + path};
  std::stringstream ss;
  ss << f.rdbuf();
  const std::string text = ss.str();
  const std::string file = path;
  Parser p(text, file);
  JVal v = p.document();
  if (v.kind != JVal::Obj) throw Fail{TAPG_EINVAL, file + ": the top level must be an object"};
  return v;
}

// -------------------------------------------------------------- accessors --

struct Doc {
  const JVal& root;
  std::string file;

  [[noreturn]] void bad(const std::string& key, const std::string& what, tapg_status code =
                                                                              TAPG_EINVAL) const {
    throw Fail{code, file + ": \"" + key + "\": " + what};
  }

  const JVal* find(const char* key) const {
    for (const auto& kv : root.obj)
      if (kv.first == key) return &kv.second;
    return nullptr;
  }

  const JVal& need(const char* key) const {
    const JVal* v = find(key);
    if (!v) throw Fail{TAPG_EINVAL, file + ": missing key \"" + key + "\""};
    return *v;
  }

  void only(std::initializer_list<const char*> keys) const {
    for (const auto& kv : root.obj) {
      bool ok = false;
      for (const char* k : keys) ok = ok || kv.first == k;
      if (!ok) throw Fail{TAPG_EINVAL, file + ": unknown key \"" + kv.first + "\""};
    }
  }

  double num(const char* key, const JVal& v) const {
    if (v.kind != JVal::Num) bad(key, std::string("expected a number, found ") + kind_name(v.kind));
    if (!std::isfinite(v.num)) bad(key, "not finite", TAPG_ENUMERIC);
    return v.num;
  }

  double num(const char* key) const { return num(key, need(key)); }

  double num_or(const char* key, double dflt) const {
    const JVal* v = find(key);
    return v ? num(key, *v) : dflt;
  }

  int integer(const char* key, const JVal& v) const {
    const double x = num(key, v);
    if (x != std::floor(x) || std::fabs(x) > 2147483647.0) bad(key, "expected an integer");
    return (int)x;
  }

  int int_or(const char* key, int dflt) const {
    const JVal* v = find(key);
    return v ? integer(key, *v) : dflt;
  }

  // Flat array of numbers; n < 0 accepts any length.
  std::vector<double> vec(const char* key, const JVal& v, long n) const {
    if (v.kind != JVal::Arr) bad(key, std::string("expected an array, found ") + kind_name(v.kind));
    if (n >= 0 && (long)v.arr.size() != n)
      bad(key, "expected " + std::to_string(n) + " entries, found " + std::to_string(v.arr.size()),
          TAPG_EDIM);
    std::vector<double> out;
    out.reserve(v.arr.size());
    for (const JVal& e : v.arr) out.push_back(num(key, e));
    return out;
  }

  std::vector<int> ivec(const char* key, const JVal& v, long n) const {
    if (v.kind != JVal::Arr) bad(key, std::string("expected an array, found ") + kind_name(v.kind));
    if (n >= 0 && (long)v.arr.size() != n)
      bad(key, "expected " + std::to_string(n) + " entries, found " + std::to_string(v.arr.size()),
          TAPG_EDIM);
    std::vector<int> out;
    out.reserve(v.arr.size());
    for (const JVal& e : v.arr) out.push_back(integer(key, e));
    return out;
  }

  // Matrix as an array of rows, returned row-major.  rows / cols < 0: taken
  // from the data (cols of an empty matrix: 0).  *r, *c receive the shape.
  std::vector<double> mat(const char* key, const JVal& v, long rows, long cols, int* r,
                          int* c) const {
    if (v.kind != JVal::Arr) bad(key, std::string("expected an array of rows, found ") +
                                          kind_name(v.kind));
    if (rows >= 0 && (long)v.arr.size() != rows)
      bad(key, "expected " + std::to_string(rows) + " rows, found " + std::to_string(v.arr.size()),
          TAPG_EDIM);
    long nc = cols;
    std::vector<double> out;
    for (size_t i = 0; i < v.arr.size(); ++i) {
      const JVal& row = v.arr[i];
      if (row.kind != JVal::Arr) bad(key, "row " + std::to_string(i) + " is not an array");
      if (nc < 0) nc = (long)row.arr.size();
      if ((long)row.arr.size() != nc)
        bad(key, "row " + std::to_string(i) + " has " + std::to_string(row.arr.size()) +
                     " entries, expected " + std::to_string(nc), TAPG_EDIM);
      for (const JVal& e : row.arr) out.push_back(num(key, e));
    }
    if (r) *r = (int)v.arr.size();
    if (c) *c = (int)(nc < 0 ? 0 : nc);
    return out;
  }

  std::string text_or(const char* key, const char* dflt) const {
    const JVal* v = find(key);
    if (!v) return dflt;
    if (v->kind != JVal::Str) bad(key, std::string("expected a string, found ") + kind_name(v->kind));
    return v->str;
  }

  bool flag_or(const char* key, bool dflt) const {
    const JVal* v = find(key);
    if (!v) return dflt;
    if (v->kind != JVal::Bool) bad(key, std::string("expected true or false, found ") +
                                            kind_name(v->kind));
    return v->b;
  }
};

template <typename F>
tapg_status guarded(F&& f) {
  try {
    clear_error();
    return f();
  } catch (const Fail& e) {
    set_error(e.msg);
    return e.code;
  } catch (const std::bad_alloc&) {
    set_error("host allocation failed");
    return TAPG_ENOMEM;
  } catch (const std::exception& e) {
    set_error(e.what());
    return TAPG_EINVAL;
  }
}

// Tree file contents: structure plus either node values or additive errors.
struct TreeFile {
  int N = 0, K = 0, nd = 0;
  std::vector<int> mu, anc;
  std::vector<double> prob;
  bool absolute = false;                // node values given directly
  std::vector<double> dem, price;       // values or errors, [K*nd] and [K]
  std::vector<int> stage;               // stage of each node
};

TreeFile read_tree(const char* path) {
  JVal root = read_json(path, "scenario tree");
  Doc d{root, path};
  d.only({"N", "nodes_per_stage", "ancestor", "probability", "children", "demand", "price",
          "demand_error", "price_error", "name", "description"});
  TreeFile t;
  t.mu = d.ivec("nodes_per_stage", d.need("nodes_per_stage"), -1);
  t.N = (int)t.mu.size();
  if (d.find("N") && d.integer("N", d.need("N")) != t.N)
    d.bad("N", "does not match the length of nodes_per_stage", TAPG_EDIM);
  if (t.N < 1) d.bad("nodes_per_stage", "at least one stage", TAPG_EDIM);
  long K = 0;
  for (int m : t.mu) {
    if (m < 1) d.bad("nodes_per_stage", "every stage has at least one node");
    K += m;
    if (K > (1L << 28)) d.bad("nodes_per_stage", "too many nodes", TAPG_EDIM);
  }
  t.K = (int)K;
  t.anc = d.ivec("ancestor", d.need("ancestor"), K);
  t.prob = d.vec("probability", d.need("probability"), K);
  t.stage.resize(K);
  for (int s = 0, n = 0; s < t.N; ++s)
    for (int q = 0; q < t.mu[s]; ++q) t.stage[n++] = s;
  if (const JVal* ch = d.find("children")) {
    // optional explicit children lists: must agree with the ancestors
    if (ch->kind != JVal::Arr) d.bad("children", "expected an array of arrays");
    std::vector<std::vector<int>> want(K);
    for (int n = 1; n < K; ++n)
      if (t.anc[n] >= 0 && t.anc[n] < K) want[t.anc[n]].push_back(n);
    const long n_inner = K - t.mu.back();
    if ((long)ch->arr.size() != K && (long)ch->arr.size() != n_inner)
      d.bad("children", "expected one list per node or per non-leaf node", TAPG_EDIM);
    for (size_t v = 0; v < ch->arr.size(); ++v) {
      const std::vector<int> got = d.ivec("children", ch->arr[v], -1);
      if (got != want[v])
        d.bad("children", "node " + std::to_string(v) + ": children disagree with \"ancestor\"");
    }
  }
  const bool has_abs = d.find("demand") || d.find("price");
  const bool has_err = d.find("demand_error") || d.find("price_error");
  if (has_abs == has_err)
    throw Fail{TAPG_EINVAL, std::string(path) + ": give either \"demand\" and \"price\" (node "
                                                "values) or \"demand_error\" and \"price_error\""};
  t.absolute = has_abs;
  const char* kd = has_abs ? "demand" : "demand_error";
  const char* kp = has_abs ? "price" : "price_error";
  int r = 0, c = 0;
  t.dem = d.mat(kd, d.need(kd), K, -1, &r, &c);
  t.nd = c;
  if (t.nd < 1) d.bad(kd, "at least one demand per node", TAPG_EDIM);
  t.price = d.vec(kp, d.need(kp), K);
  return t;
}

// Node data of a tree file, with the forecaster's nominal values added to the
// errors (eq. prediction-error: actual = forecast + error).
void node_data(const TreeFile& t, const char* tree_path, const char* fc_path,
               std::vector<double>& dem, std::vector<double>& price) {
  dem = t.dem;
  price = t.price;
  if (t.absolute) {
    if (fc_path)
      throw Fail{TAPG_EINVAL, std::string(tree_path) + ": holds node values; a forecaster "
                                                       "file is only for error trees"};
    return;
  }
  if (!fc_path)
    throw Fail{TAPG_EINVAL, std::string(tree_path) + ": holds prediction errors; a forecaster "
                                                     "file is needed"};
  JVal root = read_json(fc_path, "forecaster");
  Doc d{root, fc_path};
  d.only({"demand", "price", "name", "description"});
  const std::vector<double> fd = d.mat("demand", d.need("demand"), t.N, t.nd, nullptr, nullptr);
  const std::vector<double> fp = d.vec("price", d.need("price"), t.N);
  for (int n = 0; n < t.K; ++n) {
    const int s = t.stage[n];
    for (int i = 0; i < t.nd; ++i) dem[(size_t)n * t.nd + i] += fd[(size_t)s * t.nd + i];
    price[n] += fp[s];
  }
}

void write_num(FILE* f, double x) {
  if (std::isfinite(x)) {
    std::fprintf(f, "%.17g", x);
  } else {
    std::fputs("null", f);  // JSON has no NaN or infinity
  }
}

const char* status_name(tapg_status s) {
  switch (s) {
    case TAPG_OK: return "ok";
    case TAPG_ENOTCONV: return "not_converged";
    case TAPG_EINVAL: return "invalid_argument";
    case TAPG_EDIM: return "dimension";
    case TAPG_ENOMEM: return "out_of_memory";
    case TAPG_EDEVICE: return "device";
    case TAPG_ESTATE: return "state";
    case TAPG_ENUMERIC: return "numeric";
    default: return "unknown";
  }
}

}  // namespace

extern "C" {

tapg_status tapg_network_from_json(const char* path, tapg_network* out) {
  return guarded([&]() -> tapg_status {
    if (!out) throw Fail{TAPG_EINVAL, "network json: NULL output handle"};
    JVal root = read_json(path, "network");
    Doc d{root, path};
    d.only({"nx", "nu", "nd", "ns", "A", "B", "Gd", "E", "Ed", "xmin", "xmax", "xs", "umin",
            "umax", "name", "description"});
    int nx = 0, nu = 0, nd = 0, ns = 0, r = 0;
    const std::vector<double> A = d.mat("A", d.need("A"), -1, -1, &nx, &r);
    if (r != nx) d.bad("A", "must be square", TAPG_EDIM);
    const std::vector<double> B = d.mat("B", d.need("B"), nx, -1, nullptr, &nu);
    const std::vector<double> Gd = d.mat("Gd", d.need("Gd"), nx, -1, nullptr, &nd);
    const std::vector<double> E = d.mat("E", d.need("E"), -1, nu, &ns, nullptr);
    const std::vector<double> Ed = d.mat("Ed", d.need("Ed"), ns, ns > 0 ? nd : -1, nullptr,
                                         nullptr);
    const struct {
      const char* key;
      int val;
    } dims[] = {{"nx", nx}, {"nu", nu}, {"nd", nd}, {"ns", ns}};
    for (const auto& dm : dims)
      if (d.find(dm.key) && d.integer(dm.key, d.need(dm.key)) != dm.val)
        d.bad(dm.key, "does not match the matrices (" + std::to_string(dm.val) + ")", TAPG_EDIM);
    const std::vector<double> xmin = d.vec("xmin", d.need("xmin"), nx);
    const std::vector<double> xmax = d.vec("xmax", d.need("xmax"), nx);
    const std::vector<double> xs = d.vec("xs", d.need("xs"), nx);
    const std::vector<double> umin = d.vec("umin", d.need("umin"), nu);
    const std::vector<double> umax = d.vec("umax", d.need("umax"), nu);
    const tapg_status st = tapg_network_create(nx, nu, nd, ns, A.data(), B.data(), Gd.data(),
                                               E.data(), Ed.data(), xmin.data(), xmax.data(),
                                               xs.data(), umin.data(), umax.data(), out);
    if (st != TAPG_OK) throw Fail{st, std::string(path) + ": " + tapg_last_error()};
    return TAPG_OK;
  });
}

tapg_status tapg_tree_from_json(const char* tree_path, const char* forecaster_path,
                                tapg_tree* out) {
  return guarded([&]() -> tapg_status {
    if (!out) throw Fail{TAPG_EINVAL, "tree json: NULL output handle"};
    const TreeFile t = read_tree(tree_path);
    std::vector<double> dem, price;
    node_data(t, tree_path, forecaster_path, dem, price);
    const tapg_status st = tapg_tree_create(t.N, t.mu.data(), t.anc.data(), t.prob.data(), t.nd,
                                            dem.data(), price.data(), out);
    if (st != TAPG_OK) throw Fail{st, std::string(tree_path) + ": " + tapg_last_error()};
    return TAPG_OK;
  });
}

tapg_status tapg_tree_data_from_json(const char* tree_path, const char* forecaster_path, int K,
                                     int nd, double* demand, double* price) {
  return guarded([&]() -> tapg_status {
    if (!demand || !price) throw Fail{TAPG_EINVAL, "tree data json: NULL output array"};
    const TreeFile t = read_tree(tree_path);
    if (t.K != K || t.nd != nd)
      throw Fail{TAPG_EDIM, std::string(tree_path) + ": K = " + std::to_string(t.K) + ", nd = " +
                                std::to_string(t.nd) + "; the caller expects K = " +
                                std::to_string(K) + ", nd = " + std::to_string(nd)};
    std::vector<double> dem, pr;
    node_data(t, tree_path, forecaster_path, dem, pr);
    std::memcpy(demand, dem.data(), dem.size() * sizeof(double));
    std::memcpy(price, pr.data(), pr.size() * sizeof(double));
    return TAPG_OK;
  });
}

tapg_status tapg_config_from_json(const char* path, int nu, tapg_config* cfg, double* alpha0,
                                  double* c_energy, double* W_u) {
  return guarded([&]() -> tapg_status {
    if (!cfg || !alpha0 || !c_energy || !W_u)
      throw Fail{TAPG_EINVAL, "config json: NULL output"};
    if (nu < 1) throw Fail{TAPG_EDIM, "config json: nu >= 1"};
    JVal root = read_json(path, "controller configuration");
    Doc d{root, path};
    d.only({"W_alpha", "W_s", "W_x", "alpha0", "c_energy", "W_u", "gamma", "tol", "max_iter",
            "check_every", "precision", "power_iters", "device", "beta_rule", "averaged_primal",
            "gap_tol", "name", "description"});
    tapg_config c;
    std::memset(&c, 0, sizeof(c));
    c.W_alpha = d.num("W_alpha");
    c.W_s = d.num("W_s");
    c.W_x = d.num("W_x");
    const std::vector<double> a0 = d.vec("alpha0", d.need("alpha0"), nu);
    const std::vector<double> ce = d.vec("c_energy", d.need("c_energy"), nu);
    std::vector<double> wu((size_t)nu * nu, 0.0);
    const JVal& w = d.need("W_u");
    if (w.kind == JVal::Num) {  // a number w stands for w I
      const double s = d.num("W_u", w);
      for (int i = 0; i < nu; ++i) wu[(size_t)i * nu + i] = s;
    } else {
      wu = d.mat("W_u", w, nu, nu, nullptr, nullptr);
    }
    c.gamma = d.num_or("gamma", 0.0);
    c.tol = d.num("tol");
    c.max_iter = d.integer("max_iter", d.need("max_iter"));
    c.check_every = d.int_or("check_every", 100);
    const std::string prec = d.text_or("precision", "fp64");
    if (prec == "fp64") c.precision = TAPG_FP64;
    else if (prec == "fp32") c.precision = TAPG_FP32;
    else d.bad("precision", "expected \"fp64\" or \"fp32\"");
    c.power_iters = d.int_or("power_iters", 100);
    c.device = d.int_or("device", 0);
    c.hip_stream = nullptr;
    const std::string rule = d.text_or("beta_rule", "paper");
    if (rule == "paper") c.beta_rule = TAPG_BETA_PAPER;
    else if (rule == "simple") c.beta_rule = TAPG_BETA_SIMPLE;
    else if (rule == "zero") c.beta_rule = TAPG_BETA_ZERO;
    else d.bad("beta_rule", "expected \"paper\", \"simple\" or \"zero\"");
    c.averaged_primal = d.flag_or("averaged_primal", false) ? 1 : 0;
    c.gap_tol = d.num_or("gap_tol", 0.0);
    std::memcpy(alpha0, a0.data(), (size_t)nu * sizeof(double));
    std::memcpy(c_energy, ce.data(), (size_t)nu * sizeof(double));
    std::memcpy(W_u, wu.data(), wu.size() * sizeof(double));
    c.alpha0 = alpha0;
    c.c_energy = c_energy;
    c.W_u = W_u;
    *cfg = c;
    return TAPG_OK;
  });
}

tapg_status tapg_state_from_json(const char* path, int nx, int nu, double* x, double* u_prev) {
  return guarded([&]() -> tapg_status {
    if (!x || !u_prev) throw Fail{TAPG_EINVAL, "state json: NULL output array"};
    JVal root = read_json(path, "plant state");
    Doc d{root, path};
    d.only({"x", "u_prev", "k", "name", "description"});
    const std::vector<double> xv = d.vec("x", d.need("x"), nx);
    const std::vector<double> uv = d.vec("u_prev", d.need("u_prev"), nu);
    std::memcpy(x, xv.data(), (size_t)nx * sizeof(double));
    std::memcpy(u_prev, uv.data(), (size_t)nu * sizeof(double));
    return TAPG_OK;
  });
}

tapg_status tapg_control_output_write(const char* path, int nu, const double* u0,
                                      const tapg_result* res, tapg_status solve_status) {
  return guarded([&]() -> tapg_status {
    if (!path || !u0 || !res) throw Fail{TAPG_EINVAL, "control output: NULL argument"};
    if (nu < 1) throw Fail{TAPG_EDIM, "control output: nu >= 1"};
    const std::string tmp = std::string(path) + ".tmp";
    FILE* f = std::fopen(tmp.c_str(), "w");
    if (!f) throw Fail{TAPG_EINVAL, std::string("control output: cannot write ") + tmp};
    std::fprintf(f, "{\n  \"status\": \"%s\",\n  \"u\": [", status_name(solve_status));
    for (int i = 0; i < nu; ++i) {
      if (i) std::fputs(", ", f);
      write_num(f, u0[i]);
    }
    std::fputs("],\n", f);
    std::fprintf(f, "  \"iters\": %d,\n  \"converged\": %s,\n", res->iters,
                 res->converged ? "true" : "false");
    const struct {
      const char* key;
      double v;
    } fields[] = {{"primal_res", res->primal_res}, {"cost", res->cost},
                  {"viol_box", res->viol_box},     {"viol_eq", res->viol_eq},
                  {"gamma", res->gamma},           {"solve_ms", res->solve_ms},
                  {"dual_gap", res->dual_gap},     {"dual_obj", res->dual_obj}};
    const size_t nf = sizeof(fields) / sizeof(fields[0]);
    for (size_t k = 0; k < nf; ++k) {
      std::fprintf(f, "  \"%s\": ", fields[k].key);
      write_num(f, fields[k].v);
      std::fputs(k + 1 < nf ? ",\n" : "\n", f);
    }
    std::fputs("}\n", f);
    const bool ok = std::fflush(f) == 0 && !std::ferror(f);
    if (std::fclose(f) != 0 || !ok) {
      std::remove(tmp.c_str());
      throw Fail{TAPG_EINVAL, std::string("control output: write failed for ") + tmp};
    }
    if (std::rename(tmp.c_str(), path) != 0) {
      std::remove(tmp.c_str());
      throw Fail{TAPG_EINVAL, std::string("control output: cannot rename to ") + path};
    }
    return TAPG_OK;
  });
}

}  // extern "C"
