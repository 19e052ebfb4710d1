// Host-side check of the device geometry (decode / encode / neighbour of the
// library's native site order).  Reads "T L1 L2 L3 cstar time_bc b0 b1 b2 b3"
// on the command line and prints, for every extended-lattice site in API
// (lexicographic) order: its native index and, for mu = 0..3, the API index
// and sign of x + mu and of x - mu.
#include <cstdio>
#include <cstdlib>
#include <vector>

#include "qxd_impl.h"

using namespace qxd;

int main(int argc, char **argv) {
  if (argc != 11) return 2;
  int d[4], cstar = atoi(argv[5]), tbc = atoi(argv[6]), b[4];
  for (int m = 0; m < 4; m++) d[m] = atoi(argv[1 + m]), b[m] = atoi(argv[7 + m]);
  Geom g;
  int N[4] = {d[0], cstar ? 2 * d[1] : d[1], d[2], d[3]};
  int64_t V = 1;
  for (int m = 0; m < 4; m++) {
    g.N[m] = N[m];
    g.b[m] = b[m];
    g.nb[m] = N[m] / b[m];
    V *= N[m];
  }
  g.L1 = d[1];
  g.L1b = d[1] / b[1];
  g.shift_mask = 0;
  for (int k = 2; k <= cstar; k++) g.shift_mask |= 1 << k;
  g.time_bc = tbc;
  g.V = (int)V;
  g.Vh = (int)(V / 2);
  g.Vb = b[0] * b[1] * b[2] * b[3];
  g.Vbh = g.Vb / 2;
  g.hb3 = b[3] / 2;
  g.nblocks = g.nb[0] * g.nb[1] * g.nb[2] * g.nb[3];
  finish_geom(g);
  std::vector<int> seen(V, 0);
  std::vector<int64_t> lex_of_native(V);
  for (int i = 0; i < g.V; i++) {
    Site s = decode(g, i);
    if (encode(g, s) != i) { printf("ERR roundtrip %d\n", i); return 1; }
    int x[4];
    global_coords(g, s, x);
    for (int m = 0; m < 4; m++)
      if (x[m] < 0 || x[m] >= N[m]) { printf("ERR coords %d\n", i); return 1; }
    if (((x[0] + x[1] + x[2] + x[3]) & 1) != s.p) { printf("ERR parity %d\n", i); return 1; }
    int64_t l = ext_lex(g, x);
    if (seen[l]++) { printf("ERR not a bijection %d\n", i); return 1; }
    lex_of_native[i] = l;
  }
  std::vector<int> native_of_lex(V);
  for (int i = 0; i < g.V; i++) native_of_lex[lex_of_native[i]] = i;
  for (int64_t l = 0; l < V; l++) {
    int i = native_of_lex[l];
    Site s = decode(g, i);
    printf("%d", i);
    for (int mu = 0; mu < 4; mu++)
      for (int dir = 1; dir >= -1; dir -= 2) {
        int sg;
        Site t = neighbour(g, s, mu, dir, sg);
        int j = encode(g, t);
        if (j < 0 || j >= g.V) { printf("\nERR neighbour out of range\n"); return 1; }
        printf(" %lld %d", (long long)lex_of_native[j], sg);
      }
    printf("\n");
  }
  return 0;
}
