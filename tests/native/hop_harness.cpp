// Host-side check of the direction-generic hop (hop_generic.h) against the
// per-direction projections of hop_fwd / hop_bwd (dirac_site.h) on random
// links and spinors.  Prints the largest deviation over all directions.
#include <cmath>
#include <cstdio>
#include <random>

#include "dirac_site.h"
#include "hop_generic.h"

using namespace qxd;

int main() {
  std::mt19937_64 rng(12345);
  std::normal_distribution<double> nd;
  double worst = 0, scale = 0;
  for (int trial = 0; trial < 50; trial++)
    for (int mu = 0; mu < 4; mu++)
      for (int dir = 0; dir < 2; dir++) {
        cx<double> w[3][3], psi[4][3], a[4][3], b[4][3];
        for (auto &r : w)
          for (auto &z : r) z = {nd(rng), nd(rng)};
        for (int s = 0; s < 4; s++)
          for (int c = 0; c < 3; c++) {
            psi[s][c] = {nd(rng), nd(rng)};
            a[s][c] = b[s][c] = {nd(rng), nd(rng)};
          }
        SpinProj sp = spin_proj(mu);
        const int p1 = 5 - sp.p0;
        // accumulate onto the same starting values (b copies a's start);
        // one hop written first (INIT), a second one added on top
        cx<double> au[2][3], al[2][3], g[4][3];
        if (dir == 0) {
          hop_fwd<double>(mu, w, psi, 1.0, a);
          hop_fwd<double>(mu, w, psi, 1.0, a);
          hop_fwd<double>(mu, w, psi, 1.0, a);
          hop_generic<1, true, double>(sp, w, psi[0], psi[1], psi[sp.p0], psi[p1], au, al);
          hop_generic<1, false, double>(sp, w, psi[0], psi[1], psi[sp.p0], psi[p1], au, al);
        } else {
          hop_bwd<double>(mu, w, psi, 1.0, a);
          hop_bwd<double>(mu, w, psi, 1.0, a);
          hop_bwd<double>(mu, w, psi, 1.0, a);
          hop_generic<-1, true, double>(sp, w, psi[0], psi[1], psi[sp.p0], psi[p1], au, al);
          hop_generic<-1, false, double>(sp, w, psi[0], psi[1], psi[sp.p0], psi[p1], au, al);
        }
        lower_to_spins(sp, au, al, g);
        for (int s = 0; s < 4; s++)
          for (int c = 0; c < 3; c++) b[s][c] = b[s][c] + g[s][c];
        // the run-time direction form, with W^dag materialised for backward
        cx<double> wd[3][3];
        for (int r = 0; r < 3; r++)
          for (int c = 0; c < 3; c++) wd[r][c] = dir == 0 ? w[r][c] : conj(w[c][r]);
        hop_generic_dir<double>(sp, dir == 0 ? 1.0 : -1.0, wd, psi[0], psi[1], psi[sp.p0], psi[p1], au, al);
        lower_to_spins(sp, au, al, g);
        for (int s = 0; s < 4; s++)
          for (int c = 0; c < 3; c++) b[s][c] = b[s][c] + g[s][c];
        for (int s = 0; s < 4; s++)
          for (int c = 0; c < 3; c++) {
            worst = std::fmax(worst, std::fabs(a[s][c].re - b[s][c].re));
            worst = std::fmax(worst, std::fabs(a[s][c].im - b[s][c].im));
            scale = std::fmax(scale, std::fabs(a[s][c].re));
          }
      }
  // division by the run length of the block-major layout
  long bad = 0;
  for (uint32_t R = 1; R <= 2048; R++) {
    RunDiv d = make_rundiv(R);
    const uint32_t probes[] = {0u, 1u, R - 1, R, R + 1, 2 * R - 1, 12345677u, (1u << 31) - 1, (1u << 31) - R};
    for (uint32_t j : probes)
      if (j < (1u << 31) && d.div(j) != j / R) bad++;
    for (uint32_t j = 0; j < 3 * R + 7; j++)
      if (d.div(j) != j / R) bad++;
    std::mt19937 r32(R);
    for (int t = 0; t < 200; t++) {
      uint32_t j = r32() & 0x7fffffffu;
      if (d.div(j) != j / R) bad++;
      uint32_t e = d.base(j, 12);
      if (e != (j / R) * 12 * R + j % R) bad++;
    }
  }
  printf("%.3e %.3e %ld\n", worst, scale, bad);
  return 0;
}
