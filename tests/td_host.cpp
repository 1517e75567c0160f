// Host harness for the library's inner-product arithmetic: td_fma, td_add and
// td_round of paper_2108_10591_amd/csrc/device_common.hpp, compiled for the
// host by tests/test_td_arithmetic.py.  td_dot_grouped adds the terms in
// groups of `group` consecutive entries (forward or backward within a group),
// then combines the group totals pairwise in a tree -- the shape of the
// device's per-thread sums and block and grid reductions -- and rounds once.
#include <vector>

#include "device_common.hpp"

extern "C" double td_dot_grouped(int64_t n, const double *u, const double *v, int64_t group,
                                 int backward) {
  std::vector<ps::TD> parts;
  for (int64_t g0 = 0; g0 < n; g0 += group) {
    const int64_t g1 = g0 + group < n ? g0 + group : n;
    ps::TD t{0.0, 0.0, 0.0};
    for (int64_t j = 0; j < g1 - g0; ++j) {
      const int64_t k = backward ? g1 - 1 - j : g0 + j;
      ps::td_fma(t, u[k], v[k]);
    }
    parts.push_back(t);
  }
  while (parts.size() > 1) {
    std::vector<ps::TD> next;
    for (size_t i = 0; i < parts.size(); i += 2) {
      ps::TD t = parts[i];
      if (i + 1 < parts.size()) ps::td_add(t, parts[i + 1]);
      next.push_back(t);
    }
    parts.swap(next);
  }
  return parts.empty() ? 0.0 : ps::td_round(parts[0]);
}

extern "C" double td_round3(double a, double b, double c) {
  return ps::td_round(ps::TD{a, b, c});
}
