// Host driver that runs every exported oracle routine on small random and
// degenerate inputs, built with the address and undefined-behaviour
// sanitizers by tests/test_oracle_sanitizers.py (test infrastructure only).
#include <cmath>
#include <cstdint>
#include <cstdio>
#include <limits>
#include <random>
#include <vector>

#include "../../oracle/psdf_oracle.cpp"

int main() {
  std::mt19937 gen(7);
  std::uniform_real_distribution<double> U(-1.0, 1.0);
  // hexagon footprint, clockwise (the oracle reorders it)
  std::vector<double> fp;
  for (int k = 5; k >= 0; --k) {
    const double a = k * M_PI / 3.0;
    fp.push_back(0.5 * std::cos(a));
    fp.push_back(0.5 * std::sin(a));
  }
  const int m = 6;
  // obstacles: rectangles (closed), free segments, an open chain, an empty one
  std::vector<double> ax, ay, bx, by;
  std::vector<int32_t> off{0};
  auto add_edge = [&](double x0, double y0, double x1, double y1) {
    ax.push_back(x0); ay.push_back(y0); bx.push_back(x1); by.push_back(y1);
  };
  for (int r = 0; r < 12; ++r) {
    const double cx = 3 * U(gen), cy = 3 * U(gen), w = 0.3 + 0.2 * U(gen), h = 0.3 + 0.1 * U(gen);
    const double px[4] = {cx - w, cx + w, cx + w, cx - w}, py[4] = {cy - h, cy - h, cy + h, cy + h};
    for (int j = 0; j < 4; ++j) add_edge(px[j], py[j], px[(j + 1) % 4], py[(j + 1) % 4]);
    off.push_back((int32_t)ax.size());
  }
  for (int sgm = 0; sgm < 4; ++sgm) {
    add_edge(3 * U(gen), 3 * U(gen), 3 * U(gen), 3 * U(gen));
    off.push_back((int32_t)ax.size());
  }
  add_edge(0, 2, 1, 2.5);
  add_edge(1, 2.5, 2, 2);
  off.push_back((int32_t)ax.size());   // open two-edge chain
  off.push_back((int32_t)ax.size());   // empty obstacle
  const int M = (int)off.size() - 1, E = (int)ax.size();
  // poses: random, one at an obstacle centre (penetration), one NaN
  const int N = 9;
  std::vector<double> poses;
  for (int s = 0; s < N; ++s) {
    poses.push_back(3 * U(gen));
    poses.push_back(3 * U(gen));
    poses.push_back(M_PI * U(gen));
  }
  poses[3] = 0.5 * (ax[0] + bx[1]);
  poses[4] = 0.5 * (ay[0] + by[1]);
  poses[3 * (N - 1)] = std::numeric_limits<double>::quiet_NaN();
  std::vector<double> phi(N), grad(3 * N), sdm((size_t)N * M);
  std::vector<int32_t> obst(N), edge(N), pen(N);
  double checksum = 0.0;
  for (double eta : {1000.0, 50.0, 0.0}) {
    oracle_psdf(fp.data(), m, poses.data(), N, ax.data(), ay.data(), bx.data(), by.data(),
                off.data(), M, 1e-12, 1e-6, eta, phi.data(), obst.data(), edge.data(), grad.data(),
                pen.data(), 1);
    oracle_sd_matrix(fp.data(), m, poses.data(), N, ax.data(), ay.data(), bx.data(), by.data(),
                     off.data(), M, 1e-12, 1e-6, eta, sdm.data(), 1);
    for (int s = 0; s < N - 1; ++s) checksum += phi[s] + grad[3 * s];
    for (int i = 0; i < M; ++i) {
      const int e0 = off[i], mi = off[i + 1] - off[i];
      if (mi <= 0) continue;
      double sd, dsep, g[3], pool[16], ge[64], gf[32];
      int32_t sepd;
      oracle_obstacle(fp.data(), m, poses.data(), ax.data() + e0, ay.data() + e0, bx.data() + e0,
                      by.data() + e0, mi, 1e-12, 1e-6, eta, &sd, &sepd, &dsep, pool, g);
      oracle_obstacle_geom_grad(fp.data(), m, poses.data() + 3, ax.data() + e0, ay.data() + e0,
                                bx.data() + e0, by.data() + e0, mi, 1e-12, 1e-6, eta, ge, gf);
      checksum += sd + g[0] + ge[0] + gf[0];
    }
  }
  std::printf("ok M=%d E=%d N=%d checksum=%.6f\n", M, E, N, checksum);
  return 0;
}
