/*
 * CPU ORACLE — test infrastructure only.
 *
 * Plain, slow, obviously correct C for what the chunked speculative DFA scan
 * of Memeti & Pllana, "Analyzing large-scale DNA Sequences on Multi-core
 * Architectures" (CSE 2015), computes.  Only the test suite, the smoke check
 * and the CPU-baseline leg of the benchmark may load this file; the product
 * library never does, and this file shares no code with it.
 *
 * Contents, each with the passage of the paper it follows:
 *   - decoding of the two sequence formats (Section II: alphabet {A,C,G,T};
 *     any other byte, and a set N-mask bit, resets the automaton)
 *   - or_scan_table: the finite automaton (Q, Sigma, delta, q0, F) of Section II
 *     run sequentially from q0, reporting every visit of a final state
 *   - or_ac_build: Aho-Corasick automaton of Section II with the failure links
 *     replaced by explicit transitions ("modified AC", Section III.B.1, Fig. 2)
 *   - or_kmer_brute: the problem statement of Section II taken literally:
 *     every (overlapping) occurrence of every pattern, by direct comparison
 *   - or_regex_*: the same for a regular expression (Table IV style syntax),
 *     by Glushkov position-set simulation of Sigma* R
 *   - or_first_meet / or_kcoex: the paper's own method (Section III,
 *     Algorithm 1): equal chunks, possible starting states, a full run R0 with
 *     its per-step record, the other runs stopped at the converging point with
 *     the count fix-up, and the join that links each chunk's last state to the
 *     next chunk's first state.
 *
 * Readings of the paper taken here (the paper is silent or inconsistent):
 *   - Bytes other than A/C/G/T (either case) and N-mask bits reset the
 *     automaton to q0; no match ends on or spans such a position.
 *   - A final state may end several patterns (output set); each pattern in
 *     the set is counted.  End positions are 0-based indices of the last base,
 *     ascending, ties by ascending pattern id.
 *   - Possible starting states of chunk t>0: the image of every state under
 *     the last symbol of chunk t-1 (the first-symbol test of Algorithm 1 holds
 *     for every state of a complete DFA); a reset symbol there gives {q0}.
 *   - The last chunk takes the remainder of the division.
 *   - R0's per-step record covers `window` symbols (0 = the whole chunk); a
 *     run that has not met R0 inside the window runs to the end of its chunk.
 */
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

#define OR_RESET (-1)
#define OR_ENC_BYTE 0
#define OR_ENC_2BIT 1

/* ------------------------------------------------------------------ decode */
static int sym_of_byte(uint8_t b) {
  switch (b) {
    case 'A': case 'a': return 0;
    case 'C': case 'c': return 1;
    case 'G': case 'g': return 2;
    case 'T': case 't': return 3;
    default: return OR_RESET;
  }
}

typedef struct {
  const uint8_t* data;  /* bytes, or packed 2-bit codes */
  const uint8_t* nmask; /* 2-bit form only; may be NULL (no N) */
  uint64_t n;
  int enc;
} or_seq;

static int sym_at(const or_seq* s, uint64_t i) {
  if (s->enc == OR_ENC_BYTE) return sym_of_byte(s->data[i]);
  if (s->nmask && ((s->nmask[i >> 3] >> (i & 7)) & 1)) return OR_RESET;
  return (s->data[i >> 2] >> (2 * (i & 3))) & 3;
}

/* decode [lo, hi) into symbols (-1 = reset); exported for tests */
void or_decode(const uint8_t* data, const uint8_t* nmask, uint64_t n, int enc, uint64_t lo, uint64_t hi,
               int8_t* out) {
  or_seq s = {data, nmask, n, enc};
  for (uint64_t i = lo; i < hi; ++i) out[i - lo] = (int8_t)sym_at(&s, i);
}

/* ------------------------------------------------------------ table scan */
/*
 * Sequential run of the automaton from q0 over the whole sequence (Section II).
 * delta: uint32[n_states*4], column = symbol A,C,G,T.
 * out_off/out_ids: output sets in CSR form (ids ascending within a state).
 * counts: uint64[n_patterns] (added to).  Positions are written while
 * found < cap.  Returns the number of reported (position, pattern) events;
 * *end_state receives the state after the last base.
 */
uint64_t or_scan_table(const uint32_t* delta, uint32_t n_states, uint32_t q0, const uint32_t* out_off,
                       const uint32_t* out_ids, const uint8_t* data, const uint8_t* nmask, uint64_t n, int enc,
                       uint64_t* counts, int64_t* pos, uint32_t* pat, uint64_t cap, uint32_t* end_state) {
  or_seq sq = {data, nmask, n, enc};
  uint32_t s = q0;
  uint64_t found = 0;
  (void)n_states;
  for (uint64_t i = 0; i < n; ++i) {
    int c = sym_at(&sq, i);
    if (c == OR_RESET) { s = q0; continue; }
    s = delta[(uint64_t)s * 4 + (uint32_t)c];
    for (uint32_t k = out_off[s]; k < out_off[s + 1]; ++k) {
      counts[out_ids[k]] += 1;
      if (found < cap) { pos[found] = (int64_t)i; pat[found] = out_ids[k]; }
      ++found;
    }
  }
  if (end_state) *end_state = s;
  return found;
}

/* Same run over [lo, hi) from a given state, counting per pattern only. */
uint32_t or_run_range(const uint32_t* delta, uint32_t q0, const uint32_t* out_off, const uint32_t* out_ids,
                      const uint8_t* data, const uint8_t* nmask, uint64_t n, int enc, uint64_t lo, uint64_t hi,
                      uint32_t start, uint64_t* counts) {
  or_seq sq = {data, nmask, n, enc};
  uint32_t s = start;
  for (uint64_t i = lo; i < hi; ++i) {
    int c = sym_at(&sq, i);
    if (c == OR_RESET) { s = q0; continue; }
    s = delta[(uint64_t)s * 4 + (uint32_t)c];
    for (uint32_t k = out_off[s]; k < out_off[s + 1]; ++k) counts[out_ids[k]] += 1;
  }
  return s;
}

/* ----------------------------------------------------- Aho-Corasick (oracle's own) */
/*
 * Builds the Aho-Corasick automaton for `n_pat` patterns over {A,C,G,T}
 * (Section II) as a complete transition table (Section III.B.1: every state
 * has a transition on every symbol, so failure links disappear).
 * Patterns are NUL-terminated strings; pattern id = index.  Returns the number
 * of states, or -1 on a bad pattern (empty or a character outside ACGT), or
 * -2 if max_states is too small.  State 0 is the root (q0).
 * out_off: uint32[max_states+1]; out_ids: uint32[out_cap].
 */
int64_t or_ac_build(const char* const* pats, uint32_t n_pat, uint32_t max_states, uint32_t* delta,
                    uint32_t* out_off, uint32_t* out_ids, uint64_t out_cap) {
  /* trie with goto = -1 where absent */
  int64_t* go = (int64_t*)malloc(sizeof(int64_t) * 4 * (size_t)max_states);
  uint32_t* fail = (uint32_t*)calloc(max_states, sizeof(uint32_t));
  uint32_t* queue = (uint32_t*)malloc(sizeof(uint32_t) * (size_t)max_states);
  /* per-state output lists as linked chains of pattern ids */
  uint32_t* own_n = (uint32_t*)calloc(max_states, sizeof(uint32_t));
  uint32_t** own = (uint32_t**)calloc(max_states, sizeof(uint32_t*));
  int64_t result = 0;
  uint32_t n_states = 1;
  for (uint64_t i = 0; i < 4ull * max_states; ++i) go[i] = -1;

  for (uint32_t p = 0; p < n_pat; ++p) {
    const char* w = pats[p];
    if (!w || !w[0]) { result = -1; goto done; }
    uint32_t u = 0;
    for (const char* q = w; *q; ++q) {
      int c = sym_of_byte((uint8_t)*q);
      if (c < 0) { result = -1; goto done; }
      if (go[4 * u + c] < 0) {
        if (n_states >= max_states) { result = -2; goto done; }
        go[4 * u + c] = n_states++;
      }
      u = (uint32_t)go[4 * u + c];
    }
    own[u] = (uint32_t*)realloc(own[u], sizeof(uint32_t) * (own_n[u] + 1));
    own[u][own_n[u]++] = p;
  }

  /* breadth-first: failure function, completed transitions, output sets */
  {
    uint32_t head = 0, tail = 0;
    uint64_t n_out = 0;
    /* output set of a state = own patterns plus the output set of its failure state */
    uint32_t* outs_n = (uint32_t*)calloc(n_states, sizeof(uint32_t));
    uint32_t** outs = (uint32_t**)calloc(n_states, sizeof(uint32_t*));
    for (int a = 0; a < 4; ++a) {
      if (go[a] < 0) { delta[a] = 0; continue; }
      uint32_t v = (uint32_t)go[a];
      fail[v] = 0;
      delta[a] = v;
      queue[tail++] = v;
    }
    /* root outputs: none (patterns are non-empty) */
    outs_n[0] = 0;
    while (head < tail) {
      uint32_t u = queue[head++];
      /* outputs of u: own + outputs of fail[u] (already final: fail[u] is shallower) */
      {
        uint32_t f = fail[u];
        uint32_t k = own_n[u] + outs_n[f];
        outs[u] = (uint32_t*)malloc(sizeof(uint32_t) * (k ? k : 1));
        uint32_t m = 0;
        for (uint32_t j = 0; j < own_n[u]; ++j) outs[u][m++] = own[u][j];
        for (uint32_t j = 0; j < outs_n[f]; ++j) outs[u][m++] = outs[f][j];
        outs_n[u] = m;
      }
      for (int a = 0; a < 4; ++a) {
        if (go[4 * u + a] >= 0) {
          uint32_t v = (uint32_t)go[4 * u + a];
          fail[v] = delta[4 * fail[u] + a];
          delta[4 * u + a] = v;
          queue[tail++] = v;
        } else {
          delta[4 * u + a] = delta[4 * fail[u] + a];
        }
      }
    }
    /* CSR, ids sorted ascending */
    out_off[0] = 0;
    for (uint32_t s = 0; s < n_states; ++s) {
      uint32_t* L = outs[s];
      uint32_t k = outs_n[s];
      for (uint32_t x = 1; x < k; ++x) { /* insertion sort */
        uint32_t v = L[x];
        int64_t y = (int64_t)x - 1;
        while (y >= 0 && L[y] > v) { L[y + 1] = L[y]; --y; }
        L[y + 1] = v;
      }
      for (uint32_t x = 0; x < k; ++x) {
        if (n_out < out_cap) out_ids[n_out] = L[x];
        ++n_out;
      }
      out_off[s + 1] = (uint32_t)n_out;
    }
    for (uint32_t s = 0; s < n_states; ++s) free(outs[s]);
    free(outs);
    free(outs_n);
    if (n_out > out_cap) { result = -2; goto done; }
    result = n_states;
  }
done:
  for (uint32_t s = 0; s < max_states; ++s) free(own[s]);
  free(own);
  free(own_n);
  free(go);
  free(fail);
  free(queue);
  return result;
}

/* ------------------------------------------------------------ brute force */
/*
 * Every occurrence of every pattern, overlapping ones included (Section II),
 * by comparing the pattern against the text ending at each position.  A
 * window containing a reset symbol never matches.  Case-insensitive.
 */
uint64_t or_kmer_brute(const char* const* pats, uint32_t n_pat, const uint8_t* data, const uint8_t* nmask,
                       uint64_t n, int enc, uint64_t* counts, int64_t* pos, uint32_t* pat, uint64_t cap) {
  or_seq sq = {data, nmask, n, enc};
  uint64_t found = 0;
  uint32_t* len = (uint32_t*)malloc(sizeof(uint32_t) * (n_pat ? n_pat : 1));
  for (uint32_t p = 0; p < n_pat; ++p) len[p] = (uint32_t)strlen(pats[p]);
  for (uint64_t i = 0; i < n; ++i) {
    for (uint32_t p = 0; p < n_pat; ++p) {
      uint32_t L = len[p];
      if (L == 0 || (uint64_t)L > i + 1) continue;
      int ok = 1;
      for (uint32_t j = 0; j < L && ok; ++j) {
        int c = sym_at(&sq, i + 1 - L + j);
        if (c == OR_RESET || c != sym_of_byte((uint8_t)pats[p][j])) ok = 0;
      }
      if (ok) {
        counts[p] += 1;
        if (found < cap) { pos[found] = (int64_t)i; pat[found] = p; }
        ++found;
      }
    }
  }
  free(len);
  return found;
}

/* ---------------------------------------------------------------- regex */
/*
 * Regular expressions over {A,C,G,T} in the style of Table IV:
 *   alt    := concat ('|' concat)*
 *   concat := piece+
 *   piece  := atom ('?' | '*' | '+' | '{m}' | '{m,}' | '{m,n}')*
 *   atom   := base | '.' | '[' base+ ']' | '(' alt ')'
 * Letters are case-insensitive; '.' is any of the four bases.
 * Search semantics: position i is reported when some T[j..i] (j <= i, no
 * reset symbol inside) is in the language.  The expression must not match the
 * empty string.
 *
 * Method: Glushkov position automaton.  Every occurrence of a symbol class in
 * the expression (bounded repeats written out as copies) is a position; the
 * simulation keeps the set of positions that can have just been read.
 */
enum { RX_CLASS, RX_CAT, RX_ALT, RX_STAR, RX_OPT, RX_EMPTY };

typedef struct rx_node {
  int kind;
  int cls;              /* RX_CLASS: bit mask over A,C,G,T */
  struct rx_node* a;    /* children */
  struct rx_node* b;
  int pos;              /* RX_CLASS: position index */
} rx_node;

typedef struct {
  const char* s;
  int i;
  int err;
  rx_node** pool;
  int n_pool, cap_pool;
} rx_parser;

static rx_node* rx_new(rx_parser* P, int kind) {
  if (P->n_pool == P->cap_pool) {
    P->cap_pool = P->cap_pool ? 2 * P->cap_pool : 64;
    P->pool = (rx_node**)realloc(P->pool, sizeof(rx_node*) * (size_t)P->cap_pool);
  }
  rx_node* n = (rx_node*)calloc(1, sizeof(rx_node));
  n->kind = kind;
  n->pos = -1;
  P->pool[P->n_pool++] = n;
  return n;
}

static rx_node* rx_copy(rx_parser* P, const rx_node* t) {
  if (!t) return NULL;
  rx_node* n = rx_new(P, t->kind);
  n->cls = t->cls;
  n->a = rx_copy(P, t->a);
  n->b = rx_copy(P, t->b);
  return n;
}

static rx_node* rx_alt(rx_parser* P);

static int rx_base_bit(char c) {
  int s = sym_of_byte((uint8_t)c);
  return s < 0 ? 0 : 1 << s;
}

static rx_node* rx_atom(rx_parser* P) {
  char c = P->s[P->i];
  if (c == '(') {
    P->i++;
    rx_node* r = rx_alt(P);
    if (P->s[P->i] != ')') { P->err = 1; return r; }
    P->i++;
    return r;
  }
  if (c == '[') {
    P->i++;
    int m = 0;
    while (P->s[P->i] && P->s[P->i] != ']') {
      int b = rx_base_bit(P->s[P->i]);
      if (!b) { P->err = 1; return NULL; }
      m |= b;
      P->i++;
    }
    if (P->s[P->i] != ']' || !m) { P->err = 1; return NULL; }
    P->i++;
    rx_node* n = rx_new(P, RX_CLASS);
    n->cls = m;
    return n;
  }
  if (c == '.') {
    P->i++;
    rx_node* n = rx_new(P, RX_CLASS);
    n->cls = 15;
    return n;
  }
  int b = rx_base_bit(c);
  if (!b) { P->err = 1; return NULL; }
  P->i++;
  rx_node* n = rx_new(P, RX_CLASS);
  n->cls = b;
  return n;
}

static int rx_number(rx_parser* P, int* out) {
  int v = 0, any = 0;
  while (P->s[P->i] >= '0' && P->s[P->i] <= '9') {
    v = v * 10 + (P->s[P->i] - '0');
    if (v > 1000) { P->err = 1; return 0; }
    P->i++;
    any = 1;
  }
  *out = v;
  return any;
}

static rx_node* rx_cat2(rx_parser* P, rx_node* x, rx_node* y) {
  if (!x) return y;
  if (!y) return x;
  rx_node* n = rx_new(P, RX_CAT);
  n->a = x;
  n->b = y;
  return n;
}

/* x{m,n} = m copies of x followed by (n-m) optional copies; n < 0 means x{m,} */
static rx_node* rx_repeat(rx_parser* P, rx_node* x, int m, int n) {
  rx_node* r = NULL;
  for (int k = 0; k < m; ++k) r = rx_cat2(P, r, k == 0 ? x : rx_copy(P, x));
  if (n < 0) {
    rx_node* s = rx_new(P, RX_STAR);
    s->a = m == 0 ? x : rx_copy(P, x);
    r = rx_cat2(P, r, s);
  } else {
    for (int k = m; k < n; ++k) {
      rx_node* o = rx_new(P, RX_OPT);
      o->a = (k == 0) ? x : rx_copy(P, x);
      r = rx_cat2(P, r, o);
    }
  }
  if (!r) r = rx_new(P, RX_EMPTY);
  return r;
}

static rx_node* rx_piece(rx_parser* P) {
  rx_node* x = rx_atom(P);
  for (;;) {
    if (P->err) return x;
    char c = P->s[P->i];
    if (c == '*' || c == '+' || c == '?') {
      P->i++;
      if (c == '*') { rx_node* s = rx_new(P, RX_STAR); s->a = x; x = s; }
      else if (c == '?') { rx_node* s = rx_new(P, RX_OPT); s->a = x; x = s; }
      else x = rx_repeat(P, x, 1, -1);
    } else if (c == '{') {
      P->i++;
      int m = 0, n = 0;
      if (!rx_number(P, &m)) { P->err = 1; return x; }
      if (P->s[P->i] == '}') { n = m; }
      else if (P->s[P->i] == ',') {
        P->i++;
        if (P->s[P->i] == '}') n = -1;
        else if (!rx_number(P, &n) || n < m) { P->err = 1; return x; }
      } else { P->err = 1; return x; }
      if (P->s[P->i] != '}') { P->err = 1; return x; }
      P->i++;
      x = rx_repeat(P, x, m, n);
    } else {
      return x;
    }
  }
}

static rx_node* rx_concat(rx_parser* P) {
  rx_node* r = NULL;
  for (;;) {
    char c = P->s[P->i];
    if (!c || c == '|' || c == ')') break;
    rx_node* x = rx_piece(P);
    if (P->err) return r;
    r = rx_cat2(P, r, x);
  }
  if (!r) P->err = 1; /* empty branch */
  return r;
}

static rx_node* rx_alt(rx_parser* P) {
  rx_node* r = rx_concat(P);
  while (!P->err && P->s[P->i] == '|') {
    P->i++;
    rx_node* y = rx_concat(P);
    rx_node* n = rx_new(P, RX_ALT);
    n->a = r;
    n->b = y;
    r = n;
  }
  return r;
}

/* Glushkov sets as bit arrays of `W` 64-bit words */
typedef struct {
  int n_pos, W;
  int* cls;             /* per position class mask */
  uint64_t* first;      /* W words */
  uint64_t* last;       /* W words */
  uint64_t* follow;     /* n_pos * W words */
  int nullable;
} rx_auto;

static void rx_number_pos(rx_node* t, int* k, int* cls, int cap) {
  if (!t) return;
  if (t->kind == RX_CLASS) {
    if (*k < cap) cls[*k] = t->cls;
    t->pos = (*k)++;
    return;
  }
  rx_number_pos(t->a, k, cls, cap);
  rx_number_pos(t->b, k, cls, cap);
}

static int rx_nullable(const rx_node* t) {
  switch (t->kind) {
    case RX_CLASS: return 0;
    case RX_CAT: return rx_nullable(t->a) && rx_nullable(t->b);
    case RX_ALT: return rx_nullable(t->a) || rx_nullable(t->b);
    default: return 1; /* star, opt, empty */
  }
}

static void bs_or(uint64_t* d, const uint64_t* s, int W) { for (int i = 0; i < W; ++i) d[i] |= s[i]; }

static void rx_first(const rx_node* t, uint64_t* out, int W) {
  switch (t->kind) {
    case RX_CLASS: out[t->pos >> 6] |= 1ull << (t->pos & 63); break;
    case RX_CAT: rx_first(t->a, out, W); if (rx_nullable(t->a)) rx_first(t->b, out, W); break;
    case RX_ALT: rx_first(t->a, out, W); rx_first(t->b, out, W); break;
    case RX_STAR: case RX_OPT: rx_first(t->a, out, W); break;
    default: break;
  }
}

static void rx_last(const rx_node* t, uint64_t* out, int W) {
  switch (t->kind) {
    case RX_CLASS: out[t->pos >> 6] |= 1ull << (t->pos & 63); break;
    case RX_CAT: rx_last(t->b, out, W); if (rx_nullable(t->b)) rx_last(t->a, out, W); break;
    case RX_ALT: rx_last(t->a, out, W); rx_last(t->b, out, W); break;
    case RX_STAR: case RX_OPT: rx_last(t->a, out, W); break;
    default: break;
  }
}

/* follow(p): for CAT, last(a) -> first(b); for STAR, last(a) -> first(a) */
static void rx_follow(const rx_node* t, uint64_t* follow, int W) {
  if (!t) return;
  rx_follow(t->a, follow, W);
  rx_follow(t->b, follow, W);
  if (t->kind == RX_CAT || t->kind == RX_STAR) {
    const rx_node* from = t->a;
    const rx_node* to = t->kind == RX_CAT ? t->b : t->a;
    uint64_t* L = (uint64_t*)calloc((size_t)W, 8);
    uint64_t* F = (uint64_t*)calloc((size_t)W, 8);
    rx_last(from, L, W);
    rx_first(to, F, W);
    for (int w = 0; w < W; ++w)
      for (uint64_t m = L[w]; m; m &= m - 1) {
        int p = w * 64 + __builtin_ctzll(m);
        bs_or(follow + (size_t)p * W, F, W);
      }
    free(L);
    free(F);
  }
}

/* Parses and builds; returns an opaque handle or NULL (*err: 1 syntax, 2 nullable, 3 too big) */
void* or_regex_build(const char* text, int max_positions, int* err) {
  rx_parser P = {text, 0, 0, NULL, 0, 0};
  rx_node* root = rx_alt(&P);
  rx_auto* A = NULL;
  *err = 0;
  if (P.err || !root || P.s[P.i] != '\0') { *err = 1; goto out; }
  {
    int n_pos = 0;
    int* cls = (int*)malloc(sizeof(int) * (size_t)(max_positions > 0 ? max_positions : 1));
    rx_number_pos(root, &n_pos, cls, max_positions);
    if (n_pos > max_positions || n_pos == 0) { free(cls); *err = 3; goto out; }
    if (rx_nullable(root)) { free(cls); *err = 2; goto out; }
    A = (rx_auto*)calloc(1, sizeof(rx_auto));
    A->n_pos = n_pos;
    A->W = (n_pos + 63) / 64;
    A->cls = cls;
    A->first = (uint64_t*)calloc((size_t)A->W, 8);
    A->last = (uint64_t*)calloc((size_t)A->W, 8);
    A->follow = (uint64_t*)calloc((size_t)A->W * (size_t)n_pos, 8);
    rx_first(root, A->first, A->W);
    rx_last(root, A->last, A->W);
    rx_follow(root, A->follow, A->W);
    A->nullable = 0;
  }
out:
  for (int k = 0; k < P.n_pool; ++k) free(P.pool[k]);
  free(P.pool);
  return A;
}

int or_regex_positions(const void* h) { return ((const rx_auto*)h)->n_pos; }

void or_regex_free(void* h) {
  rx_auto* A = (rx_auto*)h;
  if (!A) return;
  free(A->cls);
  free(A->first);
  free(A->last);
  free(A->follow);
  free(A);
}

/*
 * Search run of Sigma* R: after each base, the active set is
 *   (first  union  follow(active)) restricted to positions whose class holds
 * the base; position i is reported when the active set meets `last`.
 * A reset symbol empties the active set.
 */
uint64_t or_regex_scan(const void* h, const uint8_t* data, const uint8_t* nmask, uint64_t n, int enc,
                       int64_t* pos, uint64_t cap) {
  const rx_auto* A = (const rx_auto*)h;
  or_seq sq = {data, nmask, n, enc};
  int W = A->W;
  uint64_t* act = (uint64_t*)calloc((size_t)W, 8);
  uint64_t* nxt = (uint64_t*)calloc((size_t)W, 8);
  uint64_t* cmask[4];
  uint64_t found = 0;
  for (int c = 0; c < 4; ++c) {
    cmask[c] = (uint64_t*)calloc((size_t)W, 8);
    for (int p = 0; p < A->n_pos; ++p)
      if (A->cls[p] & (1 << c)) cmask[c][p >> 6] |= 1ull << (p & 63);
  }
  for (uint64_t i = 0; i < n; ++i) {
    int c = sym_at(&sq, i);
    if (c == OR_RESET) { memset(act, 0, (size_t)W * 8); continue; }
    memcpy(nxt, A->first, (size_t)W * 8);
    for (int w = 0; w < W; ++w)
      for (uint64_t m = act[w]; m; m &= m - 1) bs_or(nxt, A->follow + (size_t)(w * 64 + __builtin_ctzll(m)) * W, W);
    int hit = 0;
    for (int w = 0; w < W; ++w) {
      act[w] = nxt[w] & cmask[c][w];
      if (act[w] & A->last[w]) hit = 1;
    }
    if (hit) {
      if (found < cap) pos[found] = (int64_t)i;
      ++found;
    }
  }
  for (int c = 0; c < 4; ++c) free(cmask[c]);
  free(act);
  free(nxt);
  return found;
}

/* ---------------------------------------------------- the paper's method */
/*
 * First index j at which two runs over the same symbols are in the same
 * state, comparing states after the same number of symbols (Section III.B.3:
 * a converging point is where runs from different states meet after the same
 * number of symbols).  Returns -1 if they never meet within n.
 */
int64_t or_first_meet(const uint32_t* r0_trace, const uint32_t* ri_trace, uint64_t n) {
  for (uint64_t j = 0; j < n; ++j)
    if (r0_trace[j] == ri_trace[j]) return (int64_t)j;
  return -1;
}

/*
 * Count fix-up at the converging point (Algorithm 1, convergence branch):
 * a run that meets R0 after j+1 symbols takes its own counts so far plus
 * R0's total minus R0's counts after the same j+1 symbols.
 */
void or_fixup(const uint64_t* own_prefix, const uint64_t* r0_total, const uint64_t* r0_prefix, uint32_t n_pat,
              uint64_t* out) {
  for (uint32_t p = 0; p < n_pat; ++p) out[p] = own_prefix[p] + r0_total[p] - r0_prefix[p];
}

/*
 * Possible starting states of a chunk whose predecessor ends with symbol c:
 * every state's successor on c, without repeats, ascending (Section III.A
 * reading: the first-symbol test is true for every state of a complete DFA).
 * A reset symbol gives {q0}.  Returns the count.
 */
uint32_t or_pss(const uint32_t* delta, uint32_t n_states, uint32_t q0, int c, uint32_t* out) {
  if (c == OR_RESET) { out[0] = q0; return 1; }
  uint8_t* seen = (uint8_t*)calloc(n_states, 1);
  uint32_t k = 0;
  for (uint32_t q = 0; q < n_states; ++q) seen[delta[(uint64_t)q * 4 + (uint32_t)c]] = 1;
  for (uint32_t q = 0; q < n_states; ++q)
    if (seen[q]) out[k++] = q;
  free(seen);
  return k;
}

/*
 * The paper's method on one CPU thread (Algorithm 1).  The sequence is cut
 * into n_chunks chunks of n / n_chunks bases (the last takes the remainder).
 * For each chunk and each possible starting state a record CR =
 * (init_state, last_state, counts[n_pat]) is produced; R0 (first candidate)
 * runs the whole chunk and records its state and counts after each of its
 * first `window` symbols (0: all symbols); every other run steps until its
 * state equals R0's state after the same number of symbols, then takes the
 * fix-up and R0's last state; a run that does not meet R0 inside the window
 * runs to the chunk end on its own.  The join then walks the chunks from q0,
 * each time picking the record whose init_state equals the previous chunk's
 * last state, and sums the counts.
 *
 * Outputs: cr_init/cr_last uint32[cap_cr], cr_counts uint64[cap_cr*n_pat],
 * cr_chunk uint32[cap_cr] (chunk of each record), totals uint64[n_pat],
 * conv_steps int64[cap_cr] (symbols consumed before stopping; -1 = R0 or no
 * convergence).  Returns the number of records, or -1 if cap_cr is too small,
 * -2 if the join finds no matching record (cannot happen for a correct PSS).
 */
int64_t or_kcoex(const uint32_t* delta, uint32_t n_states, uint32_t q0, const uint32_t* out_off,
                 const uint32_t* out_ids, uint32_t n_pat, const uint8_t* data, const uint8_t* nmask, uint64_t n,
                 int enc, uint64_t n_chunks, uint64_t window, uint32_t* cr_init, uint32_t* cr_last,
                 uint64_t* cr_counts, uint32_t* cr_chunk, int64_t* conv_steps, uint64_t cap_cr, uint64_t* totals) {
  or_seq sq = {data, nmask, n, enc};
  uint64_t base_len = n_chunks ? n / n_chunks : n;
  uint64_t n_cr = 0;
  uint32_t* pss = (uint32_t*)malloc(sizeof(uint32_t) * (n_states ? n_states : 1));
  uint64_t* fr_counts = NULL;
  uint32_t* fr_state = NULL;
  uint32_t* trace = NULL;
  uint64_t* own = (uint64_t*)calloc(n_pat ? n_pat : 1, 8);
  uint64_t* own_hist = NULL;
  int64_t rc = 0;
  if (n_chunks == 0) n_chunks = 1;

  for (uint64_t t = 0; t < n_chunks; ++t) {
    uint64_t lo = t * base_len;
    uint64_t hi = (t + 1 == n_chunks) ? n : lo + base_len;
    uint64_t len = hi - lo;
    uint64_t win = (window == 0 || window > len) ? len : window;
    uint32_t n_pss = (lo == 0) ? (pss[0] = q0, 1u) : or_pss(delta, n_states, q0, sym_at(&sq, lo - 1), pss);
    uint64_t first_cr = n_cr;
    free(fr_counts);
    free(fr_state);
    free(trace);
    free(own_hist);
    fr_counts = (uint64_t*)calloc((size_t)(win ? win : 1) * (n_pat ? n_pat : 1), 8);
    fr_state = (uint32_t*)calloc(win ? win : 1, 4);
    trace = (uint32_t*)calloc(win ? win : 1, 4);
    own_hist = (uint64_t*)calloc((size_t)(win ? win : 1) * (n_pat ? n_pat : 1), 8);
    for (uint32_t k = 0; k < n_pss; ++k) {
      uint32_t s = pss[k];
      int64_t met = -1;
      if (n_cr >= cap_cr) { rc = -1; goto done; }
      memset(own, 0, 8 * (size_t)(n_pat ? n_pat : 1));
      cr_init[n_cr] = s;
      cr_chunk[n_cr] = (uint32_t)t;
      for (uint64_t j = 0; j < len; ++j) {
        int c = sym_at(&sq, lo + j);
        s = (c == OR_RESET) ? q0 : delta[(uint64_t)s * 4 + (uint32_t)c];
        if (c != OR_RESET)
          for (uint32_t x = out_off[s]; x < out_off[s + 1]; ++x) own[out_ids[x]] += 1;
        if (j < win) {
          if (k == 0) { /* R0 records its state and counts (the per-step list) */
            fr_state[j] = s;
            memcpy(fr_counts + j * n_pat, own, 8 * (size_t)n_pat);
          } else {
            trace[j] = s;
            memcpy(own_hist + j * n_pat, own, 8 * (size_t)n_pat);
          }
        }
        if (k > 0 && j + 1 == win) {
          /* the whole window of this run is known: look for the converging point */
          met = or_first_meet(fr_state, trace, win);
          if (met >= 0) break;
        }
      }
      if (k == 0) {
        cr_last[n_cr] = s;
        memcpy(cr_counts + n_cr * n_pat, own, 8 * (size_t)n_pat);
        conv_steps[n_cr] = -1;
      } else if (met >= 0) {
        /* converged after met+1 symbols: fix-up against R0's record */
        or_fixup(own_hist + (uint64_t)met * n_pat, cr_counts + first_cr * n_pat, fr_counts + (uint64_t)met * n_pat,
                 n_pat, cr_counts + n_cr * n_pat);
        cr_last[n_cr] = cr_last[first_cr];
        conv_steps[n_cr] = met + 1;
      } else {
        /* never met R0 inside the window: ran to the end by itself */
        cr_last[n_cr] = s;
        memcpy(cr_counts + n_cr * n_pat, own, 8 * (size_t)n_pat);
        conv_steps[n_cr] = -1;
      }
      ++n_cr;
    }
  }
  /* join: link each chunk's last state to the next chunk's first state */
  {
    uint32_t cur = q0;
    uint64_t i = 0;
    for (uint32_t p = 0; p < n_pat; ++p) totals[p] = 0;
    for (uint64_t t = 0; t < n_chunks; ++t) {
      int64_t pick = -1;
      for (; i < n_cr && cr_chunk[i] == t; ++i)
        if (pick < 0 && cr_init[i] == cur) pick = (int64_t)i;
      if (pick < 0) { rc = -2; goto done; }
      for (uint32_t p = 0; p < n_pat; ++p) totals[p] += cr_counts[(uint64_t)pick * n_pat + p];
      cur = cr_last[pick];
    }
  }
  rc = (int64_t)n_cr;
done:
  free(pss);
  free(fr_counts);
  free(fr_state);
  free(trace);
  free(own);
  free(own_hist);
  return rc;
}
