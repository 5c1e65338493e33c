// Host sanitizer run of the CPU oracle (test infrastructure only).  The
// oracle's source is compiled into this driver with AddressSanitizer and
// UndefinedBehaviorSanitizer; every entry point runs on a graph read from
// stdin (int32 n, int64 m, then m sources and m destinations), error paths
// included.  One line per call: a name and the sum of what the call wrote
// (or its status), which the test compares with the oracle library built
// without sanitizers.
#include "../../oracle/probesim_oracle.cpp"

#include <cstdio>

namespace {

double sum(const std::vector<double>& v) {
  double s = 0.0;
  for (double x : v) s += x;
  return s;
}

template <class T>
bool read_all(T* p, size_t count) {
  return std::fread(p, sizeof(T), count, stdin) == count;
}

}  // namespace

int main() {
  int32_t n = 0;
  int64_t m = 0;
  if (!read_all(&n, 1) || !read_all(&m, 1) || n <= 1 || m < 0) return 2;
  std::vector<int32_t> src((size_t)m), dst((size_t)m);
  if (!read_all(src.data(), src.size()) || !read_all(dst.data(), dst.size())) return 2;

  orc_graph* g = nullptr;
  if (orc_graph_build(n, m, src.data(), dst.data(), &g) != ORC_OK) return 3;
  orc_params p{}, p0{};
  if (orc_params_derive(n, 0.6, 0.2, 0.01, -1.0, -1.0, -1.0, 0, &p) != ORC_OK) return 4;
  if (orc_params_derive(n, 0.6, 0.2, 0.01, -1.0, -1.0, 0.0, 0, &p0) != ORC_OK) return 4;
  const int32_t u = 0;
  std::vector<double> out((size_t)n);
  orc_stats st{};

  int64_t walk_nodes = 0;
  std::vector<int32_t> w((size_t)p.L);
  for (int64_t k = 0; k < 200; ++k) walk_nodes += orc_walk(g, u, k, 3, &p, w.data());
  std::printf("walks %lld\n", (long long)walk_nodes);

  for (int mode = 0; mode < 3; ++mode) {
    std::fill(out.begin(), out.end(), 0.0);
    const int rc = orc_single_source(g, u, &p, 5, 0, p.n_r, 0, mode, out.data(), &st);
    std::printf("single_source_%d %d %.17g\n", mode, rc, sum(out));
  }
  for (int f32 = 0; f32 < 2; ++f32) {
    int rc = orc_batch(g, u, &p, 7, 0, p.n_r, 1, f32, out.data(), &st);
    std::printf("batch_%d %d %.17g\n", f32, rc, sum(out));
    rc = orc_batch_hybrid(g, u, &p, 7, 0, p.n_r, 0, f32, 0.01, out.data(), &st);
    std::printf("hybrid_%d %d %.17g\n", f32, rc, sum(out));
  }
  int rc = orc_merged(g, u, &p0, 9, 0, p0.n_r, 0, out.data(), &st);
  std::printf("merged %d %.17g\n", rc, sum(out));

  const int32_t len = orc_walk(g, u, 1, 11, &p, w.data());
  if (len >= 2) {
    rc = orc_probe(g, w.data(), len, 0.6, p.eps_p, 1, out.data());
    std::printf("probe %d %.17g\n", rc, sum(out));
    rc = orc_rprobe(g, w.data(), len, 0.6, 11, 1, out.data());
    std::printf("rprobe %d %.17g\n", rc, sum(out));
  }
  int64_t hits = 0;
  rc = orc_pair_mc(g, u, 1, 0.6, 13, 0, 20000, &hits);
  std::printf("pair_mc %d %lld\n", rc, (long long)hits);
  std::vector<int32_t> tn(10);
  std::vector<double> ts(10);
  orc_batch(g, u, &p, 7, 0, p.n_r, 0, 0, out.data(), &st);
  rc = orc_topk(out.data(), n, u, 10, tn.data(), ts.data());
  std::printf("topk %d %d %.17g\n", rc, tn[0], ts[0]);

  // error paths
  orc_graph* bad = nullptr;
  const int32_t loop_s[1] = {1}, loop_d[1] = {1}, dup_s[2] = {0, 0}, dup_d[2] = {1, 1}, far_d[1] = {n};
  std::printf("err_self %d\n", orc_graph_build(n, 1, loop_s, loop_d, &bad));
  std::printf("err_dup %d\n", orc_graph_build(n, 2, dup_s, dup_d, &bad));
  std::printf("err_range %d\n", orc_graph_build(n, 1, loop_s, far_d, &bad));
  orc_params q{};
  std::printf("err_params %d\n", orc_params_derive(n, 1.5, 0.2, 0.01, -1.0, -1.0, -1.0, 0, &q));
  std::printf("err_node %d\n", orc_single_source(g, n, &p, 1, 0, p.n_r, 0, 0, out.data(), &st));
  std::printf("err_walks %d\n", orc_single_source(g, u, &p, 1, 0, p.n_r + 1, 0, 0, out.data(), &st));
  std::printf("err_merged %d\n", orc_merged(g, u, &p, 1, 0, p.n_r, 0, out.data(), &st));
  std::printf("err_topk %d\n", orc_topk(out.data(), n, u, 0, tn.data(), ts.data()));
  std::printf("err_pair %d\n", orc_pair_mc(g, u, 1, 1.0, 1, 0, 10, &hits));
  orc_graph_free(g);
  return 0;
}
