// ProbeSim CPU oracle (FP64).  TEST INFRASTRUCTURE ONLY.
//
// A plain, slow, single-threaded implementation of ProbeSim's single-source
// query, written from the paper (Liu et al., "ProbeSim: Scalable
// Single-Source and Top-k SimRank Computations on Dynamic Graphs", VLDB 2017)
// to check the GPU library against.  Only the tests, the smoke check and the
// benchmark's CPU-baseline leg may load it.  It shares no code with the GPU
// library: graph build, random numbers, walks, probes and sums are all
// written here again.
//
// What each function follows:
//   orc_params_derive   Alg. 1 (number of trials), Pruning Rule 1 (walk
//                       truncation), Theorem 2 (error split)
//   orc_philox4x32_10   Philox4x32-10 of Salmon et al., SC'11 (the paper leaves
//                       the random source open); pinned bit for bit against
//                       rocRAND's independent header-only engine
//   orc_walk            Definition of the sqrt(c)-walk (Section 2.2)
//   orc_probe           Alg. 2 (deterministic PROBE) with Pruning Rule 2, in
//                       FP64 or in the FP32 score model below
//   orc_rprobe          Alg. 4 (randomized PROBE), one run
//   orc_single_source   Alg. 1 (basic ProbeSim) with Pruning Rules 1 and 2, or
//                       with randomized PROBE (Section 4.3)
//   orc_batch           Alg. 3 (reverse reachability tree), same estimate
//   orc_batch_hybrid    Alg. 3 with the switch of Section 4.4 from
//                       deterministic to randomized PROBE
//   orc_merged          Alg. 3 with Rule 2 off, every probe of a subtree
//                       summed at the subtree's root before it is expanded
//                       (PROBE is linear in H_0, Lemma 2 / the Score
//                       equation of Section 3.3); same estimate as orc_batch
//                       at eps_p = 0
//   orc_pair_mc         Section 2.2's pairwise Monte Carlo: the fraction of
//                       pairs of sqrt(c)-walks from u and v that meet (an
//                       unbiased estimate of s(u, v), the reference of the
//                       pooled top-k evaluation on large graphs)
//   orc_topk            Definition 2 (top-k by sorting the estimates)
//
// Readings where the paper is silent or inconsistent (see the design notes):
// natural log in n_r; the squared error in n_r; the stop test is taken at every
// visited node including u_1 and a node with no in-neighbour ends the walk;
// Rule 2 removes x when Score(x) * sqrt(c)^(i-j-1) <= eps_p, for levels
// j = 0..i-2 only (never the returned level); the estimate of u itself is 1.
//
// Precision.  Rule 2 turns a floating-point comparison into a keep/remove
// decision, so besides the plain FP64 evaluation the oracle offers the FP32
// score model, in which that decision is taken in FP32: every probe score of
// an inner level is an FP32 number, each contribution of Alg. 2 is
// fl32(fl32(Score(x) * fl32(sqrt c)) * fl32(1/|I(v)|)), where fl32 is the
// nearest FP32 number; contributions are summed exactly on the grid 2^-62
// (each rounded to nearest-even there first), a level's score is that sum
// rounded to FP32, Rule 2 compares it with fl32(eps_p / sqrt(c)^(i-j-1)),
// and the returned level keeps the exact sum.  Estimates are summed over
// walks in FP64 in both modes.
//
// Randomized PROBE (Alg. 4) needs random numbers the paper leaves open:
// candidate v at iteration j of the probe of prefix (u_1..u_i) of walk k
// draws Philox4x32-10 with key (seed_lo, seed_hi ^ 0x9E3779B9) and counter
// (k, i * 2^16 + j, v, 1); words 1:0 pick its in-neighbour (as walks do) and
// word 2 < floor(sqrt(c) * 2^32) is the sqrt(c) coin.  Rule 2 does not apply
// to it (Alg. 4 has none), and each walk's probes run on their own: sharing a
// prefix saves nothing for randomized probes (Section 4.4).
//
// The switch of Section 4.4 (best of both): the probe of a tree node of
// weight w runs deterministically; before each expansion of a level H_j
// (j = 0..i-2, H_0 included), when the out-degrees of the entries Rule 2
// keeps sum to more than c0 * w * n (c0 is the caller's: the paper leaves it
// open), that probe is dropped without contributing and each of the w walks
// through the node runs randomized PROBE on the prefix instead, with the
// random numbers it draws in randomized mode.  So c0 = infinity gives the
// deterministic estimate, and with Rule 2 off c0 = 0 gives the randomized
// one (with Rule 2 on, a probe whose kept entries run out before any
// out-edge is seen stays deterministic).

#include <cmath>
#include <cstdint>
#include <cstdlib>
#include <cstring>
#include <algorithm>
#include <unordered_map>
#include <vector>

extern "C" {

typedef struct {
  int32_t n;
  int64_t m;
  int64_t* in_ptr;   // n+1 offsets into in_col
  int32_t* in_col;   // in-neighbours of each node, ascending source id
  int64_t* out_ptr;  // n+1 offsets into out_col
  int32_t* out_col;  // out-neighbours of each node, ascending target id
} orc_graph;

typedef struct {
  double c, eps_a, delta;
  double eps_s, eps_t, eps_p;  // sampling error, truncation, pruning
  int64_t n_r;                 // number of sqrt(c)-walks
  int32_t L;                   // walk truncation: keep nodes u_1..u_L
  uint32_t t_stop;             // stop when the first 32-bit word < t_stop
} orc_params;

typedef struct {
  int64_t walk_nodes;        // sum of walk lengths
  int64_t probes;            // PROBE invocations
  int64_t entries_expanded;  // frontier entries that survived Rule 2
  int64_t entries_pruned;    // frontier entries removed by Rule 2
  int64_t edges_scanned;     // out-edges looked at (excluded node included)
  int64_t next_entries;      // distinct entries created in non-final levels
  int64_t final_entries;     // entries of returned score sets
  int64_t near_threshold;    // Rule 2 tests within 1e-5 relative of eps_p
  double flip_allowance;     // sum of Score*sqrt(c)^e / n_r over those tests
  int64_t tree_nodes;        // Alg. 3 only: tree nodes below the root
  int64_t switched;          // Section 4.4 only: tree nodes whose probe switched
} orc_stats;

enum { ORC_OK = 0, ORC_EINVAL = 1, ORC_ERANGE = 2, ORC_ESELF = 3, ORC_EDUP = 4 };

// ---------------------------------------------------------------- graph ----

// Builds in- and out-adjacency from an edge list x->y (x is an in-neighbour
// of y).  The paper's graphs are simple digraphs (Section 2.1): self-loops,
// duplicates and out-of-range ids are rejected.
int orc_graph_build(int32_t n, int64_t m, const int32_t* src, const int32_t* dst,
                    orc_graph** out) {
  *out = nullptr;
  if (n <= 0 || m < 0) return ORC_EINVAL;
  std::vector<std::pair<int32_t, int32_t>> e((size_t)m);
  for (int64_t i = 0; i < m; ++i) {
    if (src[i] < 0 || src[i] >= n || dst[i] < 0 || dst[i] >= n) return ORC_ERANGE;
    if (src[i] == dst[i]) return ORC_ESELF;
    e[i] = {src[i], dst[i]};
  }
  std::sort(e.begin(), e.end());
  for (int64_t i = 1; i < m; ++i)
    if (e[i] == e[i - 1]) return ORC_EDUP;
  orc_graph* g = (orc_graph*)calloc(1, sizeof(orc_graph));
  g->n = n;
  g->m = m;
  g->in_ptr = (int64_t*)calloc((size_t)n + 1, sizeof(int64_t));
  g->out_ptr = (int64_t*)calloc((size_t)n + 1, sizeof(int64_t));
  g->in_col = (int32_t*)malloc(sizeof(int32_t) * (size_t)(m ? m : 1));
  g->out_col = (int32_t*)malloc(sizeof(int32_t) * (size_t)(m ? m : 1));
  for (auto& p : e) {
    g->out_ptr[p.first + 1]++;
    g->in_ptr[p.second + 1]++;
  }
  for (int32_t v = 0; v < n; ++v) {
    g->out_ptr[v + 1] += g->out_ptr[v];
    g->in_ptr[v + 1] += g->in_ptr[v];
  }
  std::vector<int64_t> fo(g->out_ptr, g->out_ptr + n), fi(g->in_ptr, g->in_ptr + n);
  // e is sorted by (src, dst): out-rows come out ascending by target and,
  // because sources are visited in ascending order, in-rows ascending by
  // source.
  for (auto& p : e) {
    g->out_col[fo[p.first]++] = p.second;
    g->in_col[fi[p.second]++] = p.first;
  }
  *out = g;
  return ORC_OK;
}

void orc_graph_free(orc_graph* g) {
  if (!g) return;
  free(g->in_ptr);
  free(g->in_col);
  free(g->out_ptr);
  free(g->out_col);
  free(g);
}

static inline int64_t indeg(const orc_graph* g, int32_t v) { return g->in_ptr[v + 1] - g->in_ptr[v]; }

// ----------------------------------------------------------- parameters ----

// n_r = 3c/eps^2 * ln(n/delta) (Alg. 1, first line; rounded up), walks cut to
// L = floor(ln eps_t / ln sqrt(c)) nodes (Pruning Rule 1).  The default split
// of eps_a into (eps_s, eps_t, eps_p) satisfies Theorem 2 with the optional
// eps_t/2 shift switched off:
//   eps_s = eps_a/2, eps_t = eps_a/4, eps_p = (eps_a/4)(1-sqrt c)/(1+eps_s).
// A negative override keeps the default; L_in > 0 overrides L.
int orc_params_derive(int32_t n, double c, double eps_a, double delta, double eps_s_in,
                      double eps_t_in, double eps_p_in, int32_t L_in, orc_params* p) {
  if (!(c > 0.0 && c < 1.0) || !(eps_a > 0.0 && eps_a < 1.0) || !(delta > 0.0 && delta < 1.0) ||
      n <= 0)
    return ORC_EINVAL;
  const double sc = std::sqrt(c);
  p->c = c;
  p->eps_a = eps_a;
  p->delta = delta;
  p->eps_s = eps_s_in >= 0.0 ? eps_s_in : eps_a / 2.0;
  p->eps_t = eps_t_in >= 0.0 ? eps_t_in : eps_a / 4.0;
  p->eps_p = eps_p_in >= 0.0 ? eps_p_in : (eps_a / 4.0) * (1.0 - sc) / (1.0 + p->eps_s);
  if (!(p->eps_s > 0.0) || !(p->eps_t > 0.0 && p->eps_t < 1.0)) return ORC_EINVAL;
  p->n_r = (int64_t)std::ceil(3.0 * c * std::log((double)n / delta) / (p->eps_s * p->eps_s));
  p->L = L_in > 0 ? L_in : (int32_t)std::floor(std::log(p->eps_t) / std::log(sc));
  if (p->L < 2) return ORC_EINVAL;
  p->t_stop = (uint32_t)std::floor((1.0 - sc) * 4294967296.0);
  return ORC_OK;
}

// ---------------------------------------------------------------- Philox ----

// Philox4x32 with 10 rounds.  One round maps the counter (c0,c1,c2,c3) with
// key (k0,k1) to (hi(B*c2)^c1^k0, lo(B*c2), hi(A*c0)^c3^k1, lo(A*c0)) with
// A = 0xD2511F53, B = 0xCD9E8D57; between rounds the key is advanced by the
// Weyl constants (0x9E3779B9, 0xBB67AE85).
void orc_philox4x32_10(const uint32_t ctr[4], const uint32_t key[2], uint32_t out[4]) {
  uint32_t x0 = ctr[0], x1 = ctr[1], x2 = ctr[2], x3 = ctr[3];
  uint32_t k0 = key[0], k1 = key[1];
  for (int r = 0; r < 10; ++r) {
    if (r > 0) {
      k0 += 0x9E3779B9u;
      k1 += 0xBB67AE85u;
    }
    const uint64_t pa = (uint64_t)0xD2511F53u * x0;
    const uint64_t pb = (uint64_t)0xCD9E8D57u * x2;
    const uint32_t y0 = (uint32_t)(pb >> 32) ^ x1 ^ k0;
    const uint32_t y1 = (uint32_t)pb;
    const uint32_t y2 = (uint32_t)(pa >> 32) ^ x3 ^ k1;
    const uint32_t y3 = (uint32_t)pa;
    x0 = y0;
    x1 = y1;
    x2 = y2;
    x3 = y3;
  }
  out[0] = x0;
  out[1] = x1;
  out[2] = x2;
  out[3] = x3;
}

// ----------------------------------------------------------------- walks ----

// One sqrt(c)-walk from u (Definition of the sqrt(c)-walk, Section 2.2): at
// every visited node draw one Philox block keyed by the seed with counter
// (walk k, step t, u, 0); the walk stops there when the node has no
// in-neighbour or the first word is below t_stop (probability ~ 1-sqrt c);
// otherwise it moves to the in-neighbour with index floor(r64 * |I(v)| / 2^64),
// r64 = (word2 << 32) | word1, of the ascending in-row.  Walks are cut at L
// nodes (Pruning Rule 1).  Writes the nodes, returns the length.
int32_t orc_walk(const orc_graph* g, int32_t u, int64_t k, uint64_t seed, const orc_params* p,
                 int32_t* nodes) {
  const uint32_t key[2] = {(uint32_t)seed, (uint32_t)(seed >> 32)};
  int32_t len = 0;
  int32_t v = u;
  nodes[len++] = v;
  for (uint32_t t = 0; len < p->L; ++t) {
    const uint32_t ctr[4] = {(uint32_t)k, t, (uint32_t)u, 0u};
    uint32_t w[4];
    orc_philox4x32_10(ctr, key, w);
    const int64_t d = indeg(g, v);
    if (d == 0 || w[0] < p->t_stop) break;
    const uint64_t r = ((uint64_t)w[2] << 32) | w[1];
    const uint64_t idx = (uint64_t)(((unsigned __int128)r * (uint64_t)d) >> 64);
    v = g->in_col[g->in_ptr[v] + (int64_t)idx];
    nodes[len++] = v;
  }
  return len;
}

// ----------------------------------------------------------------- probe ----

// A hash_set of (node, score) pairs as Alg. 2 uses them, kept as a dense score
// array plus the list of present keys in insertion order.
struct ScoreSet {
  std::vector<double> val;
  std::vector<char> present;
  std::vector<int32_t> keys;
  explicit ScoreSet(int32_t n) : val((size_t)n, 0.0), present((size_t)n, 0) {}
  void add(int32_t v, double x) {
    if (!present[v]) {
      present[v] = 1;
      val[v] = 0.0;
      keys.push_back(v);
    }
    val[v] += x;
  }
  void clear() {
    for (int32_t v : keys) {
      present[v] = 0;
      val[v] = 0.0;
    }
    keys.clear();
  }
};

// Alg. 2 on the partial walk path[0..i-1] = (u_1..u_i), with Pruning Rule 2
// when eps_p > 0.  H_0 = {u_i: 1}; for j = 0..i-2: remove x from H_j when
// Score(x) * sqrt(c)^(i-j-1) <= eps_p, then for each kept x and each
// out-neighbour v of x other than u_{i-j-1} add sqrt(c)/|I(v)| * Score(x) to
// H_{j+1}[v].  The returned set is H_{i-1}; by Lemma 2 (Score) its value at v
// is the first-meeting probability P(v, (u_1..u_i)).  With switch_edges >= 0
// (Section 4.4) it returns false, leaving no result, as soon as the entries
// kept at some level have more than switch_edges out-edges.
static bool probe(const orc_graph* g, const int32_t* path, int32_t i, double sc, double eps_p,
                  double n_r, double switch_edges, ScoreSet& cur, ScoreSet& nxt, std::vector<int32_t>& kept,
                  orc_stats* st) {
  cur.clear();
  cur.add(path[i - 1], 1.0);
  for (int32_t j = 0; j <= i - 2; ++j) {
    const int32_t excl = path[i - j - 2];  // u_{i-j-1}
    const double pw = std::pow(sc, (double)(i - j - 1));
    kept.clear();
    int64_t edges = 0;
    for (int32_t x : cur.keys) {
      const double s = cur.val[x];
      if (eps_p > 0.0) {
        const double proj = s * pw;
        if (st && std::fabs(proj - eps_p) <= 1e-5 * eps_p) {
          st->near_threshold++;
          st->flip_allowance += proj / n_r;
        }
        if (proj <= eps_p) {
          if (st) st->entries_pruned++;
          continue;
        }
      }
      if (st) st->entries_expanded++;
      kept.push_back(x);
      edges += g->out_ptr[x + 1] - g->out_ptr[x];
    }
    if (switch_edges >= 0.0 && (double)edges > switch_edges) return false;  // Section 4.4
    nxt.clear();
    for (int32_t x : kept) {
      const double s = cur.val[x];
      for (int64_t e = g->out_ptr[x]; e < g->out_ptr[x + 1]; ++e) {
        const int32_t v = g->out_col[e];
        if (st) st->edges_scanned++;
        if (v == excl) continue;
        nxt.add(v, sc / (double)indeg(g, v) * s);
      }
    }
    if (st && j < i - 2) st->next_entries += (int64_t)nxt.keys.size();
    std::swap(cur.val, nxt.val);
    std::swap(cur.present, nxt.present);
    std::swap(cur.keys, nxt.keys);
  }
  if (st) {
    st->probes++;
    st->final_entries += (int64_t)cur.keys.size();
  }
  return true;
}

// Exact sums on the grid 2^-62 for the FP32 score model: one 64-bit integer
// per present node (scores never exceed 1, so sums stay below 2^63).
struct FixSet {
  std::vector<int64_t> sum;
  std::vector<int32_t> keys;
  explicit FixSet(int32_t n) : sum((size_t)n, 0) {}
  void add(int32_t v, int64_t q) {
    if (sum[v] == 0) keys.push_back(v);
    sum[v] += q;
  }
  void clear() {
    for (int32_t v : keys) sum[v] = 0;
    keys.clear();
  }
};

static const double kGrid = 4611686018427387904.0;  // 2^62

// fl32(1/d) for d >= 1: of the FP32 numbers next to the double quotient, the
// one nearest to 1/d, distances |1 - r*d| compared exactly in 128-bit
// integers (r = m * 2^e with an integer mantissa m).
static float recip_f32(int64_t d) {
  const float r0 = (float)(1.0 / (double)d);
  const float cand[3] = {std::nextafter(r0, 0.0f), r0, std::nextafter(r0, 2.0f)};
  int64_t m[3];
  int e[3], emin = 0;
  for (int t = 0; t < 3; ++t) {
    const float f = std::frexp(cand[t], &e[t]);
    m[t] = (int64_t)std::ldexp(f, 24);
    e[t] -= 24;
    emin = std::min(emin, e[t]);
  }
  float best = r0;
  __int128 best_d = -1;
  for (int t = 0; t < 3; ++t) {
    // |1 - m d 2^e| * 2^-emin = |2^-emin - m d 2^(e-emin)|
    const __int128 one = (__int128)1 << (-emin);
    __int128 dist = one - ((__int128)m[t] * d << (e[t] - emin));
    if (dist < 0) dist = -dist;
    if (best_d < 0 || dist < best_d) {
      best_d = dist;
      best = cand[t];
    }
  }
  return best;
}

// fl32 of an exact grid sum
static inline float grid_to_f32(int64_t q) { return (float)q * (float)(1.0 / kGrid); }

// Alg. 2 with Rule 2 in the FP32 score model (see the header).  The returned
// set H_{i-1} keeps the exact grid sums.  switch_edges as in probe().
static bool probe_f32(const orc_graph* g, const int32_t* path, int32_t i, double c, double eps_p, double n_r,
                      double switch_edges, const std::vector<float>& inv_indeg, FixSet& cur, FixSet& nxt,
                      std::vector<int32_t>& kept, orc_stats* st) {
  const float sig = (float)std::sqrt(c);
  cur.clear();
  cur.add(path[i - 1], (int64_t)kGrid);  // H_0 = {u_i: 1}
  for (int32_t j = 0; j <= i - 2; ++j) {
    const int32_t excl = path[i - j - 2];  // u_{i-j-1}
    const float thr = eps_p > 0.0 ? (float)(eps_p / std::pow(std::sqrt(c), (double)(i - j - 1))) : 0.0f;
    kept.clear();
    int64_t edges = 0;
    for (int32_t x : cur.keys) {
      const float h = grid_to_f32(cur.sum[x]);
      if (eps_p > 0.0) {
        if (st && std::fabs((double)h - (double)thr) <= 1e-5 * (double)thr) {
          st->near_threshold++;
          st->flip_allowance += eps_p / n_r;
        }
        if (!(h > thr)) {
          if (st) st->entries_pruned++;
          continue;
        }
      }
      if (st) st->entries_expanded++;
      kept.push_back(x);
      edges += g->out_ptr[x + 1] - g->out_ptr[x];
    }
    if (switch_edges >= 0.0 && (double)edges > switch_edges) return false;  // Section 4.4
    nxt.clear();
    for (int32_t x : kept) {
      const float a = grid_to_f32(cur.sum[x]) * sig;
      for (int64_t e = g->out_ptr[x]; e < g->out_ptr[x + 1]; ++e) {
        const int32_t v = g->out_col[e];
        if (st) st->edges_scanned++;
        if (v == excl) continue;
        const float contrib = a * inv_indeg[v];
        const int64_t q = std::llrint((double)contrib * kGrid);
        if (q != 0) nxt.add(v, q);
      }
    }
    if (st && j < i - 2) st->next_entries += (int64_t)nxt.keys.size();
    std::swap(cur.sum, nxt.sum);
    std::swap(cur.keys, nxt.keys);
  }
  if (st) {
    st->probes++;
    st->final_entries += (int64_t)cur.keys.size();
  }
  return true;
}

// One probe in either precision; adds weight * Score(v) to acc.  Returns
// false, adding nothing, when the probe switched (switch_edges as in probe()).
struct Prober {
  const orc_graph* g;
  bool f32;
  ScoreSet cur, nxt;
  FixSet fcur, fnxt;
  std::vector<int32_t> kept;
  std::vector<float> inv;  // fl32(1/|I(v)|), FP32 model only
  Prober(const orc_graph* g_, bool f) : g(g_), f32(f), cur(f ? 1 : g_->n), nxt(f ? 1 : g_->n),
                                        fcur(f ? g_->n : 1), fnxt(f ? g_->n : 1) {
    if (f32) {
      inv.assign((size_t)g->n, 0.0f);
      for (int32_t v = 0; v < g->n; ++v)
        if (indeg(g, v) > 0) inv[v] = recip_f32(indeg(g, v));
    }
  }
  bool run(const int32_t* path, int32_t i, double c, double eps_p, double n_r_over_w, double w,
           std::vector<double>& acc, orc_stats* st, double switch_edges = -1.0) {
    if (f32) {
      if (!probe_f32(g, path, i, c, eps_p, n_r_over_w, switch_edges, inv, fcur, fnxt, kept, st)) return false;
      for (int32_t v : fcur.keys) acc[v] += w * ((double)fcur.sum[v] / kGrid);
    } else {
      if (!probe(g, path, i, std::sqrt(c), eps_p, n_r_over_w, switch_edges, cur, nxt, kept, st)) return false;
      for (int32_t v : cur.keys) acc[v] += w * cur.val[v];
    }
    return true;
  }
};

// Alg. 4 on the partial walk path[0..i-1] = (u_1..u_i) of walk k: returns
// H_{i-1} as the list `cur` (membership flags in `in`, cleared on return).
static void rprobe(const orc_graph* g, const int32_t* path, int32_t i, double c, uint64_t seed, int64_t k,
                   std::vector<int32_t>& cur, std::vector<int32_t>& cand, std::vector<char>& in,
                   std::vector<char>& seen, orc_stats* st) {
  const uint32_t key[2] = {(uint32_t)seed, (uint32_t)(seed >> 32) ^ 0x9E3779B9u};
  const uint32_t t_sc = (uint32_t)std::floor(std::sqrt(c) * 4294967296.0);
  cur.assign(1, path[i - 1]);
  in[path[i - 1]] = 1;
  std::vector<int32_t> nxt;
  for (int32_t j = 0; j <= i - 2; ++j) {
    const int32_t excl = path[i - j - 2];  // u_{i-j-1}
    cand.clear();
    for (int32_t x : cur)
      for (int64_t e = g->out_ptr[x]; e < g->out_ptr[x + 1]; ++e) {
        const int32_t v = g->out_col[e];
        if (st) st->edges_scanned++;
        if (v == excl || seen[v]) continue;
        seen[v] = 1;
        cand.push_back(v);
      }
    nxt.clear();
    for (int32_t v : cand) {
      seen[v] = 0;
      const uint32_t ctr[4] = {(uint32_t)k, ((uint32_t)i << 16) | (uint32_t)j, (uint32_t)v, 1u};
      uint32_t w[4];
      orc_philox4x32_10(ctr, key, w);
      const uint64_t r = ((uint64_t)w[1] << 32) | w[0];
      const int64_t d = indeg(g, v);  // >= 1: v has an in-neighbour in cur
      const int32_t x = g->in_col[g->in_ptr[v] + (int64_t)(((unsigned __int128)r * (uint64_t)d) >> 64)];
      if (in[x] && w[2] < t_sc) nxt.push_back(v);
    }
    for (int32_t x : cur) in[x] = 0;
    cur.swap(nxt);
    for (int32_t x : cur) in[x] = 1;
    if (st) st->next_entries += (int64_t)cur.size();
  }
  for (int32_t x : cur) in[x] = 0;
  if (st) {
    st->probes++;
    st->final_entries += (int64_t)cur.size();
  }
}

// Alg. 4 alone, for tests: 1 for the nodes of H_{i-1}, else 0.
int orc_rprobe(const orc_graph* g, const int32_t* path, int32_t i, double c, uint64_t seed, int64_t k,
               double* out) {
  if (i < 2) return ORC_EINVAL;
  for (int32_t t = 0; t < i; ++t)
    if (path[t] < 0 || path[t] >= g->n) return ORC_ERANGE;
  std::vector<int32_t> cur, cand;
  std::vector<char> in((size_t)g->n, 0), seen((size_t)g->n, 0);
  rprobe(g, path, i, c, seed, k, cur, cand, in, seen, nullptr);
  std::fill(out, out + g->n, 0.0);
  for (int32_t v : cur) out[v] = 1.0;
  return ORC_OK;
}

// Alg. 2 alone, for tests: dense scores of PROBE((u_1..u_i)).
int orc_probe(const orc_graph* g, const int32_t* path, int32_t i, double c, double eps_p, int f32,
              double* out) {
  if (i < 2) return ORC_EINVAL;
  for (int32_t t = 0; t < i; ++t)
    if (path[t] < 0 || path[t] >= g->n) return ORC_ERANGE;
  std::vector<double> acc((size_t)g->n, 0.0);
  Prober pr(g, f32 != 0);
  pr.run(path, i, c, eps_p, 1.0, 1.0, acc, nullptr);
  std::copy(acc.begin(), acc.end(), out);
  return ORC_OK;
}

static void finish(const orc_graph* g, int32_t u, const orc_params* p, int bias_shift,
                   const std::vector<double>& acc, double* out) {
  for (int32_t v = 0; v < g->n; ++v) {
    out[v] = acc[v] / (double)p->n_r;
    if (bias_shift && v != u) out[v] += p->eps_t / 2.0;  // Section 4.1, after Rule 1
  }
  out[u] = 1.0;
}

// Alg. 1: for walks k in [k_begin, k_end) sample W_k(u), PROBE every prefix
// (u_1..u_i), i = 2..len, and sum the scores; the estimate is the sum over
// walks divided by n_r (the running average of Alg. 1 is the same number).
// A sub-range of walks gives that range's share of the sum.
// mode: bit 0 the FP32 score model, bit 1 randomized PROBE (Alg. 4).
int orc_single_source(const orc_graph* g, int32_t u, const orc_params* p, uint64_t seed,
                      int64_t k_begin, int64_t k_end, int bias_shift, int mode, double* out, orc_stats* st) {
  if (u < 0 || u >= g->n) return ORC_ERANGE;
  if (k_begin < 0 || k_end > p->n_r || k_begin > k_end) return ORC_EINVAL;
  if (st) memset(st, 0, sizeof(*st));
  std::vector<double> acc((size_t)g->n, 0.0);
  std::vector<int32_t> walk((size_t)p->L);
  if (mode & 2) {
    std::vector<int32_t> cur, cand;
    std::vector<char> in((size_t)g->n, 0), seen((size_t)g->n, 0);
    for (int64_t k = k_begin; k < k_end; ++k) {
      const int32_t len = orc_walk(g, u, k, seed, p, walk.data());
      if (st) st->walk_nodes += len;
      for (int32_t i = 2; i <= len; ++i) {
        rprobe(g, walk.data(), i, p->c, seed, k, cur, cand, in, seen, st);
        for (int32_t v : cur) acc[v] += 1.0;
      }
    }
    finish(g, u, p, bias_shift, acc, out);
    return ORC_OK;
  }
  Prober pr(g, (mode & 1) != 0);
  for (int64_t k = k_begin; k < k_end; ++k) {
    const int32_t len = orc_walk(g, u, k, seed, p, walk.data());
    if (st) st->walk_nodes += len;
    for (int32_t i = 2; i <= len; ++i) pr.run(walk.data(), i, p->c, p->eps_p, (double)p->n_r, 1.0, acc, st);
  }
  finish(g, u, p, bias_shift, acc, out);
  return ORC_OK;
}

// Alg. 3: insert the walks into a reverse reachability tree (one tree node per
// distinct prefix (u_1..u_q), q >= 2, weighted by the number of walks sharing
// it), PROBE every tree node once and add weight/n_r * Score.  With c0 >= 0
// the probe of a node of weight w switches as Section 4.4 describes (see the
// header): the node's walks then probe its prefix with Alg. 4, adding 1 per
// returned node, each with its own random numbers.
static int batch(const orc_graph* g, int32_t u, const orc_params* p, uint64_t seed, int64_t k_begin,
                 int64_t k_end, int bias_shift, int f32, double c0, double* out, orc_stats* st) {
  if (u < 0 || u >= g->n) return ORC_ERANGE;
  if (k_begin < 0 || k_end > p->n_r || k_begin > k_end) return ORC_EINVAL;
  if (st) memset(st, 0, sizeof(*st));
  struct TNode {
    int64_t parent;
    int32_t node, depth;
    int64_t weight;
    std::vector<int64_t> walks;  // the walks through the node (Section 4.4 only)
  };
  const bool hybrid = c0 >= 0.0;
  std::vector<TNode> tree;
  tree.push_back({-1, u, 1, 0, {}});
  std::unordered_map<uint64_t, int64_t> child;  // (parent id, graph node) -> id
  std::vector<int32_t> walk((size_t)p->L);
  for (int64_t k = k_begin; k < k_end; ++k) {
    const int32_t len = orc_walk(g, u, k, seed, p, walk.data());
    if (st) st->walk_nodes += len;
    int64_t cur = 0;
    for (int32_t i = 2; i <= len; ++i) {
      const uint64_t key = ((uint64_t)cur << 32) | (uint32_t)walk[i - 1];
      auto it = child.find(key);
      if (it == child.end()) {
        tree.push_back({cur, walk[i - 1], i, 0, {}});
        it = child.emplace(key, (int64_t)tree.size() - 1).first;
      }
      cur = it->second;
      tree[cur].weight++;
      if (hybrid) tree[cur].walks.push_back(k);
    }
  }
  if (st) st->tree_nodes = (int64_t)tree.size() - 1;
  std::vector<double> acc((size_t)g->n, 0.0);
  std::vector<int32_t> path;
  Prober pr(g, (f32 & 1) != 0);
  std::vector<int32_t> rcur, rcand;
  std::vector<char> in(hybrid ? (size_t)g->n : 0, 0), seen(hybrid ? (size_t)g->n : 0, 0);
  for (size_t q = 1; q < tree.size(); ++q) {
    const int32_t i = tree[q].depth;
    path.assign((size_t)i, 0);
    for (int64_t a = (int64_t)q; a >= 0; a = tree[a].parent) path[tree[a].depth - 1] = tree[a].node;
    const double w = (double)tree[q].weight;
    const double switch_edges = hybrid ? c0 * w * (double)g->n : -1.0;
    if (pr.run(path.data(), i, p->c, p->eps_p, (double)p->n_r / w, w, acc, st, switch_edges)) continue;
    if (st) st->switched++;
    for (int64_t k : tree[q].walks) {
      rprobe(g, path.data(), i, p->c, seed, k, rcur, rcand, in, seen, st);
      for (int32_t v : rcur) acc[v] += 1.0;
    }
  }
  finish(g, u, p, bias_shift, acc, out);
  return ORC_OK;
}

int orc_batch(const orc_graph* g, int32_t u, const orc_params* p, uint64_t seed, int64_t k_begin,
              int64_t k_end, int bias_shift, int f32, double* out, orc_stats* st) {
  if (f32 & 2)  // randomized probes are per walk: the tree changes nothing
    return orc_single_source(g, u, p, seed, k_begin, k_end, bias_shift, f32, out, st);
  return batch(g, u, p, seed, k_begin, k_end, bias_shift, f32, -1.0, out, st);
}

// Alg. 3 with the switch of Section 4.4 at constant c0 >= 0 (f32: bit 0 as in
// orc_single_source).
int orc_batch_hybrid(const orc_graph* g, int32_t u, const orc_params* p, uint64_t seed, int64_t k_begin,
                     int64_t k_end, int bias_shift, int f32, double c0, double* out, orc_stats* st) {
  if (!(c0 >= 0.0)) return ORC_EINVAL;
  return batch(g, u, p, seed, k_begin, k_end, bias_shift, f32 & 1, c0, out, st);
}

// Merged probing over the reverse reachability tree (Rule 2 off).  A probe
// of the tree node (u_1..u_i) applies, to H_0 = e_{u_i}, the level maps
// T_{i-1}, ..., T_1, where T_p sends a score set at walk position p+1 to
// position p: T_p(H)[v] = sum over x in H with v in O(x), v != u_p, of
// sqrt(c)/|I(v)| * H[x].  T_p depends on the walk prefix only through u_p,
// the node of the tree ancestor at depth p, and every T_p is linear, so the
// weighted probes of a subtree can be added before they are pushed through
// the maps they share:  X(t) = w(t) e_{node(t)} + sum over the children c of
// t of T_{depth(t)}(X(c)), for the tree nodes t below the root, and the
// estimate is X(root) / n_r (the root itself is not probed).  Nodes are taken
// deepest first; each node's set is expanded once, along its tree edge.
// Rule 2 prunes per probe and has no merged form, so eps_p must be 0.
int orc_merged(const orc_graph* g, int32_t u, const orc_params* p, uint64_t seed, int64_t k_begin, int64_t k_end,
               int bias_shift, double* out, orc_stats* st) {
  if (u < 0 || u >= g->n) return ORC_ERANGE;
  if (k_begin < 0 || k_end > p->n_r || k_begin > k_end || p->eps_p != 0.0) return ORC_EINVAL;
  if (st) memset(st, 0, sizeof(*st));
  std::vector<int64_t> parent(1, -1), weight(1, 0);
  std::vector<int32_t> node(1, u), depth(1, 1);
  std::unordered_map<uint64_t, int64_t> child;  // (parent id, graph node) -> id
  std::vector<int32_t> walk((size_t)p->L);
  int32_t max_depth = 1;
  for (int64_t k = k_begin; k < k_end; ++k) {
    const int32_t len = orc_walk(g, u, k, seed, p, walk.data());
    if (st) st->walk_nodes += len;
    int64_t cur = 0;
    for (int32_t i = 2; i <= len; ++i) {
      const uint64_t key = ((uint64_t)cur << 32) | (uint32_t)walk[i - 1];
      auto it = child.find(key);
      if (it == child.end()) {
        parent.push_back(cur);
        node.push_back(walk[i - 1]);
        depth.push_back(i);
        weight.push_back(0);
        it = child.emplace(key, (int64_t)node.size() - 1).first;
      }
      cur = it->second;
      weight[cur]++;
      max_depth = std::max(max_depth, i);
    }
  }
  const int64_t count = (int64_t)node.size();
  if (st) st->tree_nodes = count - 1;
  std::vector<std::vector<int64_t>> by_depth((size_t)max_depth + 1);
  for (int64_t t = 1; t < count; ++t) by_depth[(size_t)depth[t]].push_back(t);
  std::vector<std::unordered_map<int32_t, double>> X((size_t)count);
  const double sc = std::sqrt(p->c);
  for (int32_t d = max_depth; d >= 2; --d) {
    for (int64_t t : by_depth[(size_t)d]) {
      X[(size_t)t][node[t]] += (double)weight[t];  // the node's own probe
      const int64_t a = parent[t];
      const int32_t excl = node[a];                 // u at walk position d - 1
      auto& up = X[(size_t)a];
      for (const auto& xv : X[(size_t)t]) {
        const int32_t x = xv.first;
        if (st) st->entries_expanded++;
        for (int64_t e = g->out_ptr[x]; e < g->out_ptr[x + 1]; ++e) {
          const int32_t v = g->out_col[e];
          if (st) st->edges_scanned++;
          if (v == excl) continue;
          up[v] += sc / (double)indeg(g, v) * xv.second;
        }
      }
      if (st) st->probes++;
      std::unordered_map<int32_t, double>().swap(X[(size_t)t]);
    }
  }
  std::vector<double> acc((size_t)g->n, 0.0);
  for (const auto& xv : X[0]) acc[(size_t)xv.first] = xv.second;
  if (st) st->final_entries = (int64_t)X[0].size();
  finish(g, u, p, bias_shift, acc, out);
  return ORC_OK;
}

// Pairwise Monte Carlo (Section 2.2, the baseline the paper compares with):
// s(u, v) is the probability that a sqrt(c)-walk from u and one from v meet,
// that is, stand on the same node after the same number of steps.  Sample k
// runs the two walks in lockstep.  At step t each walk draws its own Philox
// block, key (seed_lo, seed_hi ^ v), counter (k_lo, k_hi, t, side) with side
// 0 for the walk from u and 1 for the walk from v; the walk stops when its
// node has no in-neighbour or word 0 is below floor((1 - sqrt c) 2^32), else
// it moves to the in-neighbour that words 2:1 pick, as in orc_walk.  The
// sample ends when either walk stops, and counts a meeting when both move
// onto the same node.  Walks are not truncated, so the fraction of samples
// that meet is an unbiased estimate of s(u, v) itself.  Writes the meetings
// among samples [k_begin, k_end); every sample meets when u = v.
int orc_pair_mc(const orc_graph* g, int32_t u, int32_t v, double c, uint64_t seed, int64_t k_begin,
                int64_t k_end, int64_t* hits) {
  if (u < 0 || u >= g->n || v < 0 || v >= g->n) return ORC_ERANGE;
  if (!(c > 0.0 && c < 1.0) || k_begin < 0 || k_end < k_begin) return ORC_EINVAL;
  if (u == v) {
    *hits = k_end - k_begin;
    return ORC_OK;
  }
  const uint32_t t_stop = (uint32_t)std::floor((1.0 - std::sqrt(c)) * 4294967296.0);
  const uint32_t key[2] = {(uint32_t)seed, (uint32_t)(seed >> 32) ^ (uint32_t)v};
  int64_t met = 0;
  for (int64_t k = k_begin; k < k_end; ++k) {
    int32_t x[2] = {u, v};
    for (uint32_t t = 0;; ++t) {
      bool stop = false;
      for (uint32_t side = 0; side < 2 && !stop; ++side) {
        const uint32_t ctr[4] = {(uint32_t)k, (uint32_t)((uint64_t)k >> 32), t, side};
        uint32_t w[4];
        orc_philox4x32_10(ctr, key, w);
        const int64_t d = indeg(g, x[side]);
        if (d == 0 || w[0] < t_stop) {
          stop = true;
          break;
        }
        const uint64_t r = ((uint64_t)w[2] << 32) | w[1];
        const uint64_t idx = (uint64_t)(((unsigned __int128)r * (uint64_t)d) >> 64);
        x[side] = g->in_col[g->in_ptr[x[side]] + (int64_t)idx];
      }
      if (stop) break;
      if (x[0] == x[1]) {
        ++met;
        break;
      }
    }
  }
  *hits = met;
  return ORC_OK;
}

// Definition 2: the k nodes v != u with the largest estimates; equal
// estimates are ordered by ascending node id.  k must lie in [1, n-1].
int orc_topk(const double* s, int32_t n, int32_t u, int32_t k, int32_t* nodes, double* scores) {
  if (u < 0 || u >= n) return ORC_ERANGE;
  if (k < 1 || k > n - 1) return ORC_EINVAL;
  std::vector<int32_t> ids;
  ids.reserve((size_t)n - 1);
  for (int32_t v = 0; v < n; ++v)
    if (v != u) ids.push_back(v);
  std::sort(ids.begin(), ids.end(), [&](int32_t a, int32_t b) {
    if (s[a] != s[b]) return s[a] > s[b];
    return a < b;
  });
  for (int32_t t = 0; t < k; ++t) {
    nodes[t] = ids[t];
    scores[t] = s[ids[t]];
  }
  return ORC_OK;
}

}  // extern "C"
