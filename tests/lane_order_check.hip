// Host check of the compile-time pencil lane order (TaskOrder): for every
// axis, the order is a permutation of the pencil tasks, and within every
// aligned group of G lanes (G = the layout's read and write widths) the
// first nodes are distinct modulo G, so that each pencil access is served
// without bank conflicts.  Prints one line per (configuration, axis) with
// the number of groups that break each constraint; exits nonzero unless the
// 3D Euler N=4 float64 order is a permutation that meets the write
// constraints (8 and 16 lanes) and the 16-byte read constraint everywhere.
#include <cstdio>

#include "../paper_1801_08682_amd/csrc/pde.hpp"
#include "../paper_1801_08682_amd/csrc/kernels_fwd.hpp"

template <class K, int ns, int I>
int check(const char* name) {
  constexpr int T = ns * K::NF, s = adg::ipow(K::n, I);
  static constexpr auto o = adg::make_task_order<K, ns, I>();
  // permutation: every natural first node appears exactly once
  bool ok = true;
  for (int task = 0; task < T; ++task) {
    const int tt = task / K::NF, b = task % K::NF;
    const int off = tt * K::NSP + K::slot((b % s) + s * K::n * (b / s));
    int hits = 0;
    for (int lane = 0; lane < T; ++lane) hits += (o.e0[lane] == off);
    ok = ok && hits == 1;
  }
  int broken[3] = {0, 0, 0};
  for (int c = 0; c < K::NGROUP; ++c) {
    const int G = K::group(c);
    for (int g0 = 0; g0 < T; g0 += G) {
      bool dup = false;
      for (int x = g0; x < g0 + G && x < T; ++x)
        for (int y = x + 1; y < g0 + G && y < T; ++y)
          if (o.e0[x] % G == o.e0[y] % G) dup = true;
      broken[c] += dup;
    }
  }
  std::printf("%s ns=%d I=%d permutation=%d broken groups (G=%d,%d,%d): %d %d %d\n", name, ns, I,
              ok ? 1 : 0, K::group(0), K::NGROUP > 1 ? K::group(1) : 0,
              K::NGROUP > 2 ? K::group(2) : 0, broken[0], broken[1], broken[2]);
  // the constraints before the last: write widths and the 16-byte read width
  int strict = 0;
  for (int c = 0; c + 1 < K::NGROUP; ++c) strict += broken[c];
  return ok ? strict : 1000000;
}

template <class K>
int all_axes(const char* name) {
  return check<K, K::S, 0>(name) + check<K, K::S, 1>(name) + check<K, K::S, 2>(name);
}

int main() {
  using namespace adg;
  const int c2 = all_axes<Fwd<3, 4, Euler, double>>("euler3d_n4_double");
  all_axes<Fwd<3, 4, Euler, float>>("euler3d_n4_float");
  all_axes<Fwd<3, 3, Acoustic, double>>("acoustic3d_n3_double");
  all_axes<Fwd<3, 5, Elastic, double>>("elastic3d_n5_double");
  all_axes<Fwd<3, 7, Euler, double>>("euler3d_n7_double");
  std::printf("euler3d_n4_double strict_broken=%d\n", c2);
  return c2 == 0 ? 0 : 1;
}
