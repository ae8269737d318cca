// Automaton compilers and analysis (host side of libcoex).
//
//  - compile_kmers: Aho-Corasick automaton (Section II of the paper) whose
//    failure transitions are replaced by explicit ones so that every state has
//    a successor on every symbol (Section III.B.1, Fig. 2), then minimised with
//    the output sets as labels.
//  - compile_regex: regular expression (Table IV syntax) -> Thompson NFA ->
//    subset construction of the search automaton Sigma* R -> minimisation.
//  - from_table: a caller-supplied quintuple (Section II), validated.
//  - analyze: dense accepting index, largest output set, synchronising depth
//    (pair graph), and the possible-starting-state tables for k-base
//    lookbacks (Section III.A, generalised from the paper's single symbol).
#include <algorithm>
#include <array>
#include <cstring>
#include <deque>
#include <map>
#include <unordered_map>

#include "coex.h"
#include "dfa.hpp"

namespace coex {

namespace {

int sym_code(char ch) {
  switch (ch) {
    case 'A': case 'a': return 0;
    case 'C': case 'c': return 1;
    case 'G': case 'g': return 2;
    case 'T': case 't': return 3;
    default: return -1;
  }
}

// Moore partition refinement.  `label[s]` is an initial class key (states
// with different labels are never merged).  Returns the minimal automaton
// restricted to states reachable from q0, numbered breadth-first from q0.
void minimise(const std::vector<uint32_t>& delta, const std::vector<uint32_t>& label, uint32_t q0,
              std::vector<uint32_t>& new_delta, std::vector<uint32_t>& rep_of_class, uint32_t& new_q0) {
  const uint32_t n = (uint32_t)label.size();
  // reachable states
  std::vector<uint8_t> reach(n, 0);
  std::vector<uint32_t> order;
  order.push_back(q0);
  reach[q0] = 1;
  for (size_t i = 0; i < order.size(); ++i)
    for (int c = 0; c < 4; ++c) {
      uint32_t t = delta[order[i] * 4 + c];
      if (!reach[t]) { reach[t] = 1; order.push_back(t); }
    }
  std::vector<uint32_t> cls(n, 0);
  {
    std::map<uint32_t, uint32_t> ids;
    for (uint32_t s : order) {
      auto it = ids.find(label[s]);
      if (it == ids.end()) it = ids.emplace(label[s], (uint32_t)ids.size()).first;
      cls[s] = it->second;
    }
  }
  uint32_t n_cls = 0;
  for (uint32_t s : order) n_cls = std::max(n_cls, cls[s] + 1);
  for (;;) {
    std::map<std::array<uint32_t, 5>, uint32_t> sig;
    std::vector<uint32_t> next(n, 0);
    for (uint32_t s : order) {
      std::array<uint32_t, 5> key = {cls[s], cls[delta[s * 4]], cls[delta[s * 4 + 1]], cls[delta[s * 4 + 2]],
                                     cls[delta[s * 4 + 3]]};
      auto it = sig.find(key);
      if (it == sig.end()) it = sig.emplace(key, (uint32_t)sig.size()).first;
      next[s] = it->second;
    }
    uint32_t m = (uint32_t)sig.size();
    cls.swap(next);
    if (m == n_cls) break;
    n_cls = m;
  }
  // number classes breadth-first from q0's class
  std::vector<int64_t> num(n_cls, -1);
  std::vector<uint32_t> rep;  // representative state per new number
  std::deque<uint32_t> q;
  num[cls[q0]] = 0;
  rep.push_back(q0);
  q.push_back(q0);
  while (!q.empty()) {
    uint32_t s = q.front();
    q.pop_front();
    for (int c = 0; c < 4; ++c) {
      uint32_t t = delta[s * 4 + c];
      if (num[cls[t]] < 0) {
        num[cls[t]] = (int64_t)rep.size();
        rep.push_back(t);
        q.push_back(t);
      }
    }
  }
  new_delta.assign(rep.size() * 4, 0);
  for (size_t i = 0; i < rep.size(); ++i)
    for (int c = 0; c < 4; ++c) new_delta[i * 4 + c] = (uint32_t)num[cls[delta[rep[i] * 4 + c]]];
  rep_of_class = rep;
  new_q0 = 0;
}

}  // namespace

// ------------------------------------------------------------------ k-mers
int compile_kmers(const std::vector<std::string>& kmers, std::unique_ptr<Dfa>& out) {
  if (kmers.empty()) return COEX_EINVAL;
  size_t total = 0;
  for (const auto& w : kmers) {
    if (w.empty()) return COEX_EALPHABET;
    for (char ch : w)
      if (sym_code(ch) < 0) return COEX_EALPHABET;
    total += w.size();
  }
  // keyword tree
  struct Node { int32_t child[4]; int32_t fail; std::vector<uint32_t> own; };
  std::vector<Node> tree;
  tree.reserve(total + 1);
  tree.push_back(Node{{-1, -1, -1, -1}, 0, {}});
  for (uint32_t id = 0; id < kmers.size(); ++id) {
    int32_t u = 0;
    for (char ch : kmers[id]) {
      int c = sym_code(ch);
      if (tree[u].child[c] < 0) {
        tree[u].child[c] = (int32_t)tree.size();
        tree.push_back(Node{{-1, -1, -1, -1}, 0, {}});
      }
      u = tree[u].child[c];
    }
    tree[u].own.push_back(id);
  }
  const uint32_t n = (uint32_t)tree.size();
  // failure links breadth-first; complete transitions: missing edges follow
  // the failure state's (already complete) transition
  std::vector<uint32_t> delta(n * 4, 0);
  std::vector<std::vector<uint32_t>> outs(n);
  std::vector<uint32_t> bfs;
  bfs.reserve(n);
  for (int c = 0; c < 4; ++c) {
    int32_t v = tree[0].child[c];
    delta[c] = v < 0 ? 0u : (uint32_t)v;
    if (v >= 0) { tree[v].fail = 0; bfs.push_back((uint32_t)v); }
  }
  for (size_t i = 0; i < bfs.size(); ++i) {
    uint32_t u = bfs[i];
    outs[u] = tree[u].own;
    const auto& fo = outs[tree[u].fail];
    outs[u].insert(outs[u].end(), fo.begin(), fo.end());
    std::sort(outs[u].begin(), outs[u].end());
    for (int c = 0; c < 4; ++c) {
      int32_t v = tree[u].child[c];
      if (v >= 0) {
        tree[v].fail = (int32_t)delta[tree[u].fail * 4 + c];
        delta[u * 4 + c] = (uint32_t)v;
        bfs.push_back((uint32_t)v);
      } else {
        delta[u * 4 + c] = delta[tree[u].fail * 4 + c];
      }
    }
  }
  // minimise with the output sets as labels
  std::map<std::vector<uint32_t>, uint32_t> label_ids;
  std::vector<uint32_t> label(n);
  for (uint32_t s = 0; s < n; ++s) {
    auto it = label_ids.find(outs[s]);
    if (it == label_ids.end()) it = label_ids.emplace(outs[s], (uint32_t)label_ids.size()).first;
    label[s] = it->second;
  }
  std::vector<uint32_t> nd, rep;
  uint32_t q0 = 0;
  minimise(delta, label, 0, nd, rep, q0);
  if (rep.size() > kMaxStates) return COEX_ETOOBIG;
  auto d = std::make_unique<Dfa>();
  d->n_states = (uint32_t)rep.size();
  d->q0 = q0;
  d->n_patterns = (uint32_t)kmers.size();
  d->delta = std::move(nd);
  d->out_off.assign(d->n_states + 1, 0);
  for (uint32_t s = 0; s < d->n_states; ++s) {
    const auto& o = outs[rep[s]];
    d->out_ids.insert(d->out_ids.end(), o.begin(), o.end());
    d->out_off[s + 1] = (uint32_t)d->out_ids.size();
  }
  analyze(*d);
  out = std::move(d);
  return COEX_OK;
}

// ------------------------------------------------------------------ regex
namespace {

struct RNode {
  enum Kind { CLS, CAT, ALT, REP } kind;
  uint8_t cls = 0;
  int lo = 0, hi = 0;  // REP: {lo, hi}, hi < 0 = unbounded
  std::vector<std::unique_ptr<RNode>> kids;
};

struct RParser {
  const std::string& s;
  size_t i = 0;
  bool bad = false;
  explicit RParser(const std::string& str) : s(str) {}
  char peek() const { return i < s.size() ? s[i] : '\0'; }

  std::unique_ptr<RNode> alt() {
    auto first = cat();
    if (bad) return first;
    if (peek() != '|') return first;
    auto n = std::make_unique<RNode>();
    n->kind = RNode::ALT;
    n->kids.push_back(std::move(first));
    while (!bad && peek() == '|') {
      ++i;
      n->kids.push_back(cat());
    }
    return n;
  }
  std::unique_ptr<RNode> cat() {
    auto n = std::make_unique<RNode>();
    n->kind = RNode::CAT;
    while (!bad) {
      char c = peek();
      if (c == '\0' || c == '|' || c == ')') break;
      n->kids.push_back(piece());
    }
    if (n->kids.empty()) bad = true;
    return n;
  }
  bool number(int& v) {
    size_t st = i;
    v = 0;
    while (i < s.size() && s[i] >= '0' && s[i] <= '9') {
      v = v * 10 + (s[i] - '0');
      if (v > 1000) { bad = true; return false; }
      ++i;
    }
    return i > st;
  }
  std::unique_ptr<RNode> piece() {
    auto a = atom();
    while (!bad) {
      char c = peek();
      int lo, hi;
      if (c == '*') { lo = 0; hi = -1; ++i; }
      else if (c == '+') { lo = 1; hi = -1; ++i; }
      else if (c == '?') { lo = 0; hi = 1; ++i; }
      else if (c == '{') {
        ++i;
        if (!number(lo)) { bad = true; break; }
        if (peek() == '}') { hi = lo; }
        else if (peek() == ',') {
          ++i;
          if (peek() == '}') hi = -1;
          else if (!number(hi) || hi < lo) { bad = true; break; }
        } else { bad = true; break; }
        if (peek() != '}') { bad = true; break; }
        ++i;
      } else break;
      auto r = std::make_unique<RNode>();
      r->kind = RNode::REP;
      r->lo = lo;
      r->hi = hi;
      r->kids.push_back(std::move(a));
      a = std::move(r);
    }
    return a;
  }
  std::unique_ptr<RNode> atom() {
    auto n = std::make_unique<RNode>();
    n->kind = RNode::CLS;
    char c = peek();
    if (c == '(') {
      ++i;
      auto inner = alt();
      if (peek() != ')') bad = true; else ++i;
      return inner;
    }
    if (c == '[') {
      ++i;
      while (!bad && peek() != ']') {
        int k = sym_code(peek());
        if (k < 0) { bad = true; break; }
        n->cls |= (uint8_t)(1u << k);
        ++i;
      }
      if (peek() != ']' || n->cls == 0) bad = true; else ++i;
      return n;
    }
    if (c == '.') { ++i; n->cls = 15; return n; }
    int k = sym_code(c);
    if (k < 0) { bad = true; return n; }
    ++i;
    n->cls = (uint8_t)(1u << k);
    return n;
  }
};

// Thompson NFA: each state has at most one symbol edge (class + target) and
// any number of epsilon edges.
struct Nfa {
  std::vector<uint8_t> cls;
  std::vector<int32_t> to;
  std::vector<std::vector<int32_t>> eps;
  int32_t add() {
    cls.push_back(0);
    to.push_back(-1);
    eps.emplace_back();
    return (int32_t)cls.size() - 1;
  }
};

struct Frag { int32_t in, out; };

bool build_nfa(const RNode* t, Nfa& A, Frag& f, size_t limit) {
  if (A.cls.size() > limit) return false;
  switch (t->kind) {
    case RNode::CLS: {
      f.in = A.add();
      f.out = A.add();
      A.cls[f.in] = t->cls;
      A.to[f.in] = f.out;
      return true;
    }
    case RNode::CAT: {
      f.in = f.out = A.add();
      for (const auto& k : t->kids) {
        Frag g;
        if (!build_nfa(k.get(), A, g, limit)) return false;
        A.eps[f.out].push_back(g.in);
        f.out = g.out;
      }
      return true;
    }
    case RNode::ALT: {
      f.in = A.add();
      f.out = A.add();
      for (const auto& k : t->kids) {
        Frag g;
        if (!build_nfa(k.get(), A, g, limit)) return false;
        A.eps[f.in].push_back(g.in);
        A.eps[g.out].push_back(f.out);
      }
      return true;
    }
    case RNode::REP: {
      // x{lo,hi}: lo mandatory copies, then hi-lo optional copies (or a loop)
      f.in = f.out = A.add();
      for (int k = 0; k < t->lo; ++k) {
        Frag g;
        if (!build_nfa(t->kids[0].get(), A, g, limit)) return false;
        A.eps[f.out].push_back(g.in);
        f.out = g.out;
      }
      if (t->hi < 0) {
        Frag g;
        if (!build_nfa(t->kids[0].get(), A, g, limit)) return false;
        int32_t end = A.add();
        A.eps[f.out].push_back(g.in);
        A.eps[f.out].push_back(end);
        A.eps[g.out].push_back(g.in);
        A.eps[g.out].push_back(end);
        f.out = end;
      } else {
        int32_t end = A.add();
        for (int k = t->lo; k < t->hi; ++k) {
          Frag g;
          if (!build_nfa(t->kids[0].get(), A, g, limit)) return false;
          A.eps[f.out].push_back(g.in);
          A.eps[f.out].push_back(end);
          f.out = g.out;
        }
        A.eps[f.out].push_back(end);
        f.out = end;
      }
      return true;
    }
  }
  return false;
}

void closure(const Nfa& A, std::vector<int32_t>& set, std::vector<uint32_t>& mark, uint32_t stamp) {
  for (size_t i = 0; i < set.size(); ++i) {
    int32_t s = set[i];
    for (int32_t t : A.eps[s])
      if (mark[t] != stamp) { mark[t] = stamp; set.push_back(t); }
  }
}

}  // namespace

int compile_regex(const std::string& regex, std::unique_ptr<Dfa>& out) {
  RParser P(regex);
  auto root = P.alt();
  if (P.bad || P.i != regex.size()) return COEX_ESYNTAX;
  Nfa A;
  Frag f;
  if (!build_nfa(root.get(), A, f, 200000)) return COEX_ETOOBIG;
  const int32_t fin = f.out;
  const size_t nn = A.cls.size();
  std::vector<uint32_t> mark(nn, 0);
  uint32_t stamp = 0;
  // start closure (included in every subset: search semantics)
  std::vector<int32_t> start = {f.in};
  mark[f.in] = ++stamp;
  closure(A, start, mark, stamp);
  for (int32_t s : start)
    if (s == fin) return COEX_ESYNTAX;  // matches the empty string
  // subset key: sorted states carrying a symbol edge, plus the final flag
  auto key_of = [&](const std::vector<int32_t>& set) {
    std::vector<int32_t> k;
    bool acc = false;
    for (int32_t s : set) {
      if (A.cls[s]) k.push_back(s);
      if (s == fin) acc = true;
    }
    std::sort(k.begin(), k.end());
    k.push_back(acc ? -1 : -2);
    return k;
  };
  std::map<std::vector<int32_t>, uint32_t> ids;
  std::vector<std::vector<int32_t>> sets;
  std::vector<uint32_t> delta;
  std::vector<uint32_t> accepting;
  auto intern = [&](const std::vector<int32_t>& set) -> int64_t {
    auto k = key_of(set);
    auto it = ids.find(k);
    if (it != ids.end()) return it->second;
    if (sets.size() >= 16 * kMaxStates) return -1;
    uint32_t id = (uint32_t)sets.size();
    ids.emplace(k, id);
    sets.push_back(k);  // the key already lists the symbol-edge states
    accepting.push_back(k.back() == -1 ? 1u : 0u);
    delta.resize(sets.size() * 4, 0);
    return id;
  };
  if (intern(start) < 0) return COEX_ETOOBIG;
  for (size_t di = 0; di < sets.size(); ++di) {
    for (int c = 0; c < 4; ++c) {
      std::vector<int32_t> nx = start;
      ++stamp;
      for (int32_t s : nx) mark[s] = stamp;
      for (int32_t s : sets[di]) {
        if (s < 0) continue;
        if ((A.cls[s] >> c) & 1) {
          int32_t t = A.to[s];
          if (mark[t] != stamp) { mark[t] = stamp; nx.push_back(t); }
        }
      }
      closure(A, nx, mark, stamp);
      int64_t id = intern(nx);
      if (id < 0) return COEX_ETOOBIG;
      delta[di * 4 + c] = (uint32_t)id;
    }
  }
  std::vector<uint32_t> nd, rep;
  uint32_t q0 = 0;
  minimise(delta, accepting, 0, nd, rep, q0);
  if (rep.size() > kMaxStates) return COEX_ETOOBIG;
  auto d = std::make_unique<Dfa>();
  d->n_states = (uint32_t)rep.size();
  d->q0 = q0;
  d->n_patterns = 1;
  d->delta = std::move(nd);
  d->out_off.assign(d->n_states + 1, 0);
  for (uint32_t s = 0; s < d->n_states; ++s) {
    if (accepting[rep[s]]) d->out_ids.push_back(0);
    d->out_off[s + 1] = (uint32_t)d->out_ids.size();
  }
  analyze(*d);
  out = std::move(d);
  return COEX_OK;
}

// ------------------------------------------------------------------ table
int from_table(const uint32_t* delta, uint32_t n_states, uint32_t q0, const uint32_t* out_off,
               const uint32_t* out_ids, uint32_t n_patterns, std::unique_ptr<Dfa>& out) {
  if (!delta || !out_off || n_states == 0 || q0 >= n_states) return COEX_EINVAL;
  if (n_states > kMaxStates) return COEX_ETOOBIG;
  if (out_off[0] != 0) return COEX_EINVAL;
  for (uint32_t s = 0; s < n_states; ++s)
    if (out_off[s + 1] < out_off[s]) return COEX_EINVAL;
  if (out_off[n_states] > 0 && !out_ids) return COEX_EINVAL;
  for (uint64_t i = 0; i < (uint64_t)n_states * 4; ++i)
    if (delta[i] >= n_states) return COEX_EINVAL;
  auto d = std::make_unique<Dfa>();
  d->n_states = n_states;
  d->q0 = q0;
  d->n_patterns = n_patterns;
  d->delta.assign(delta, delta + (size_t)n_states * 4);
  d->out_off.assign(out_off, out_off + n_states + 1);
  d->out_ids.assign(out_ids, out_ids + out_off[n_states]);
  for (uint32_t s = 0; s < n_states; ++s) {
    auto b = d->out_ids.begin() + out_off[s], e = d->out_ids.begin() + out_off[s + 1];
    std::sort(b, e);
    for (auto it = b; it != e; ++it) {
      if (*it >= n_patterns) return COEX_EINVAL;
      if (it + 1 != e && *(it + 1) == *it) return COEX_EINVAL;
    }
  }
  analyze(*d);
  out = std::move(d);
  return COEX_OK;
}

// ------------------------------------------------------------------ analysis
namespace {

// Longest run of symbols two distinct states can read without meeting: the
// longest path in the graph of unordered state pairs whose successors stay
// distinct.  sync depth = that + 1, or kNoSync when the graph has a cycle.
uint32_t sync_depth(const Dfa& d) {
  const uint64_t n = d.n_states;
  if (n <= 1) return 0;
  auto idx = [n](uint64_t p, uint64_t q) -> uint64_t {  // p < q
    return p * n - p * (p + 1) / 2 + (q - p - 1);
  };
  const uint64_t np = n * (n - 1) / 2;
  std::vector<uint8_t> color(np, 0);   // 0 new, 1 on stack, 2 done
  std::vector<uint32_t> longest(np, 0);
  struct Fr { uint32_t p, q; uint8_t c; };
  std::vector<Fr> st;
  uint32_t best = 0;
  for (uint32_t p0 = 0; p0 < n; ++p0)
    for (uint32_t q0 = p0 + 1; q0 < n; ++q0) {
      if (color[idx(p0, q0)]) continue;
      st.push_back({p0, q0, 0});
      color[idx(p0, q0)] = 1;
      while (!st.empty()) {
        Fr& fr = st.back();
        if (fr.c < 4) {
          uint32_t a = d.delta[fr.p * 4 + fr.c], b = d.delta[fr.q * 4 + fr.c];
          ++fr.c;
          if (a == b) continue;
          if (a > b) std::swap(a, b);
          uint64_t j = idx(a, b);
          if (color[j] == 1) return kNoSync;  // cycle: some pair never meets
          if (color[j] == 0) { color[j] = 1; st.push_back({a, b, 0}); }
          continue;
        }
        // all successors finished
        uint32_t L = 0;
        for (int c = 0; c < 4; ++c) {
          uint32_t a = d.delta[fr.p * 4 + c], b = d.delta[fr.q * 4 + c];
          if (a == b) continue;
          if (a > b) std::swap(a, b);
          L = std::max(L, longest[idx(a, b)] + 1);
        }
        uint64_t j = idx(fr.p, fr.q);
        longest[j] = L;
        color[j] = 2;
        best = std::max(best, L);
        st.pop_back();
      }
    }
  return best + 1;
}

}  // namespace

void analyze(Dfa& d) {
  const uint32_t n = d.n_states;
  d.acc_index.assign(n, -1);
  d.acc_state.clear();
  d.max_out = 0;
  for (uint32_t s = 0; s < n; ++s) {
    uint32_t w = d.out_off[s + 1] - d.out_off[s];
    if (w) {
      d.acc_index[s] = (int32_t)d.acc_state.size();
      d.acc_state.push_back(s);
    }
    d.max_out = std::max(d.max_out, w);
  }
  d.n_accepting = (uint32_t)d.acc_state.size();
  d.sync_depth = sync_depth(d);
  {
    // 3 * 8192 symbols of a linear congruential generator (Numerical
    // Recipes constants, top two bits), run from q0
    uint32_t s = d.q0, x = 12345u, hits = 0;
    constexpr uint32_t kSteps = 8192;
    for (uint32_t i = 0; i < kSteps; ++i) {
      bool hit = false;
      for (int j = 0; j < 3; ++j) {
        x = x * 1664525u + 1013904223u;
        s = d.delta[s * 4 + (x >> 30)];
        hit |= d.acc_index[s] >= 0;
      }
      hits += hit ? 1u : 0u;
    }
    d.match_density = (double)hits / kSteps;
  }
  // possible starting states after a k-base lookback: image of Q under the
  // k-gram, sorted; built level by level (append the newest symbol)
  std::vector<std::vector<uint16_t>> prev(1);
  prev[0].resize(n);
  for (uint32_t s = 0; s < n; ++s) prev[0][s] = (uint16_t)s;
  std::vector<uint32_t> seen(n, 0);
  uint32_t stamp = 0;
  for (uint32_t k = 1; k <= kMaxLookback; ++k) {
    const uint64_t m_prev = prev.size();
    std::vector<std::vector<uint16_t>> cur(m_prev * 4);
    for (uint32_t c = 0; c < 4; ++c)
      for (uint64_t w = 0; w < m_prev; ++w) {
        auto& out = cur[w + c * m_prev];
        ++stamp;
        for (uint16_t s : prev[w]) {
          uint32_t t = d.delta[(uint32_t)s * 4 + c];
          if (seen[t] != stamp) { seen[t] = stamp; out.push_back((uint16_t)t); }
        }
        std::sort(out.begin(), out.end());
      }
    PssTable& T = d.pss[k];
    T.k = k;
    T.off.assign(cur.size() + 1, 0);
    T.states.clear();
    T.max_size = 0;
    for (size_t w = 0; w < cur.size(); ++w) {
      T.states.insert(T.states.end(), cur[w].begin(), cur[w].end());
      T.off[w + 1] = (uint32_t)T.states.size();
      T.max_size = std::max<uint32_t>(T.max_size, (uint32_t)cur[w].size());
    }
    prev.swap(cur);
  }
}

}  // namespace coex
