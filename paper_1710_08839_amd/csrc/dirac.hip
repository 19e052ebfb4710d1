// Wilson-clover operator kernels: full D, hopping part, Pauli term, and the
// two half-lattice passes of the even-odd Schur complement (Sec. 2.4):
//   odd pass   t_o = D_oo^-1 (self_o + c * acc(in_e))
//   even pass  out_e = P self_e + c * acc(t_o)      (or self_e + c acc)
// so that D^ psi_e = P_e psi_e + acc(t_o)/2 with t_o = -D_oo^-1 acc(psi_e)/2.
// One thread per site; every operand is a structure-of-arrays field in native
// order, so the 64 lanes of a wavefront read consecutive sites.
#include <map>
#include <mutex>
#include <tuple>

#include "dirac_site.h"
#include "launch.h"

namespace qxd {

namespace {

template <int P, int KIND, int GROUP>
__global__ void __launch_bounds__(256) dirac_kernel(Geom g, const typename St<P>::pair_t *links,
                                                    const typename St<P>::real_t *angles, int qhat,
                                                    const typename St<P>::pair_t *pauli,
                                                    const typename St<P>::pair_t *pinv,
                                                    Spinor<P> in, Spinor<P> self, Spinor<P> out,
                                                    typename St<P>::comp_t c) {
  using T = typename St<P>::comp_t;
  // A work-group owns whole lattice blocks (both parities for the full-lattice
  // kinds, one parity for the half-lattice passes), in XCD-aware order, so
  // that the even/odd neighbours of a site and the blocks next to it are read
  // through the same L2.
  constexpr bool half = KIND == DK_ODD || KIND == DK_EVEN || KIND == DK_EVEN_ID;
  const int per_block = half ? g.Vbh : 2 * g.Vbh;
  const int wg = xcd_order(blockIdx.x, gridDim.x);
  int blk, r;
  if (per_block <= (int)blockDim.x) {  // whole blocks per work-group
    const int bpw = blockDim.x / per_block;
    blk = wg * bpw + threadIdx.x / per_block;
    r = threadIdx.x % per_block;
  } else {                             // a block spread over several work-groups
    const int wpb = per_block / blockDim.x;
    blk = wg / wpb;
    r = (wg % wpb) * blockDim.x + threadIdx.x;
  }
  if (blk >= g.nblocks) return;
  int par = half ? (KIND == DK_ODD ? 1 : 0) : (r >= g.Vbh);
  int i = par * g.Vh + blk * g.Vbh + (r >= g.Vbh ? r - g.Vbh : r);
  cx<T> res[4][3];
  if (KIND != DK_PAULI) {
    Site s = decode(g, i);
    hop_sum<P, T, GROUP>(g, links, angles, qhat, in, s, i, res);
#pragma unroll
    for (int a = 0; a < 4; a++)
#pragma unroll
      for (int b = 0; b < 3; b++) res[a][b] = c * res[a][b];
  } else {
#pragma unroll
    for (int a = 0; a < 4; a++)
#pragma unroll
      for (int b = 0; b < 3; b++) res[a][b] = {0, 0};
  }
  if (KIND == DK_FULL || KIND == DK_PAULI || KIND == DK_EVEN) {
    cx<T> v[4][3], pv[4][3];
    load_spinor<P, T>(self, i, v);
    pauli_mul<P, T>(pauli, g.V, i, v, pv);
#pragma unroll
    for (int a = 0; a < 4; a++)
#pragma unroll
      for (int b = 0; b < 3; b++) res[a][b] = res[a][b] + pv[a][b];
  } else if (KIND == DK_EVEN_ID || KIND == DK_ODD) {
    if (self.data != nullptr) {
      cx<T> v[4][3];
      load_spinor<P, T>(self, i, v);
#pragma unroll
      for (int a = 0; a < 4; a++)
#pragma unroll
        for (int b = 0; b < 3; b++) res[a][b] = res[a][b] + v[a][b];
    }
  }
  if (KIND == DK_ODD) {
    cx<T> pv[4][3];
    pauli_mul<P, T>(pinv, g.Vh, i - g.Vh, res, pv);
    store_spinor<P, T>(out, i, pv);
  } else {
    store_spinor<P, T>(out, i, res);
  }
}

template <int P, int KIND, int G>
void launch_k(unsigned gr, int threads, hipStream_t st, const Geom &g, const typename St<P>::pair_t *links,
              const typename St<P>::real_t *angles, int qhat, const typename St<P>::pair_t *pauli,
              const typename St<P>::pair_t *pinv, Spinor<P> vin, Spinor<P> vself, Spinor<P> vout,
              typename St<P>::comp_t c) {
  dirac_kernel<P, KIND, G><<<gr, threads, 0, st>>>(g, links, angles, qhat, pauli, pinv, vin, vself, vout, c);
}

template <int P, int KIND>
void launch_g(int group, unsigned gr, int threads, hipStream_t st, const Geom &g, const typename St<P>::pair_t *links,
              const typename St<P>::real_t *angles, int qhat, const typename St<P>::pair_t *pauli,
              const typename St<P>::pair_t *pinv, Spinor<P> vin, Spinor<P> vself, Spinor<P> vout,
              typename St<P>::comp_t c) {
  switch (group) {
    case 1: launch_k<P, KIND, 1>(gr, threads, st, g, links, angles, qhat, pauli, pinv, vin, vself, vout, c); break;
    case 4: launch_k<P, KIND, 4>(gr, threads, st, g, links, angles, qhat, pauli, pinv, vin, vself, vout, c); break;
    case 8: launch_k<P, KIND, 8>(gr, threads, st, g, links, angles, qhat, pauli, pinv, vin, vself, vout, c); break;
    default: launch_k<P, KIND, 2>(gr, threads, st, g, links, angles, qhat, pauli, pinv, vin, vself, vout, c); break;
  }
}

template <int P>
hipError_t launch_p(DiracKind kind, int group, const Geom &g, const OpFields &f, SpinorArg in,
                    SpinorArg self, SpinorArg out, double c, hipStream_t st) {
  using pt = typename St<P>::pair_t;
  using rt = typename St<P>::real_t;
  using T = typename St<P>::comp_t;
  auto links = (const pt *)f.links;
  auto angles = (const rt *)f.angles;
  auto pauli = (const pt *)f.pauli;
  auto pinv = (const pt *)f.pinv;
  Spinor<P> vin = spinor_view<P>(in.ptr, in.sites, in.off);
  Spinor<P> vself = self.ptr ? spinor_view<P>(self.ptr, self.sites, self.off) : Spinor<P>{nullptr, nullptr, 0, 0};
  Spinor<P> vout = spinor_view<P>(out.ptr, out.sites, out.off);
  // work-group size: whole blocks, about 256 threads
  bool half = kind == DK_ODD || kind == DK_EVEN || kind == DK_EVEN_ID;
  int per_block = half ? g.Vbh : 2 * g.Vbh;
  int threads;
  unsigned gr;
  if (per_block <= 256) {
    int bpw = 256 / per_block;
    threads = bpw * per_block;
    gr = grid_for(g.nblocks, bpw);
  } else {
    // block sites are a multiple of 16, so per_block is a multiple of 8: use
    // the largest power-of-two divisor of per_block up to 256 threads
    threads = 256;
    while (per_block % threads) threads >>= 1;
    gr = (unsigned)g.nblocks * (per_block / threads);
  }
  T cc = (T)c;
  switch (kind) {
    case DK_FULL: launch_g<P, DK_FULL>(group, gr, threads, st, g, links, angles, f.qhat, pauli, pinv, vin, vself, vout, cc); break;
    case DK_HOP: launch_g<P, DK_HOP>(group, gr, threads, st, g, links, angles, f.qhat, pauli, pinv, vin, vself, vout, cc); break;
    case DK_PAULI: launch_g<P, DK_PAULI>(1, gr, threads, st, g, links, angles, f.qhat, pauli, pinv, vin, vself, vout, cc); break;
    case DK_ODD: launch_g<P, DK_ODD>(group, gr, threads, st, g, links, angles, f.qhat, pauli, pinv, vin, vself, vout, cc); break;
    case DK_EVEN: launch_g<P, DK_EVEN>(group, gr, threads, st, g, links, angles, f.qhat, pauli, pinv, vin, vself, vout, cc); break;
    case DK_EVEN_ID: launch_g<P, DK_EVEN_ID>(group, gr, threads, st, g, links, angles, f.qhat, pauli, pinv, vin, vself, vout, cc); break;
  }
  return hipGetLastError();
}

hipError_t launch_any(int prec, DiracKind kind, int group, const Geom &g, const OpFields &f, SpinorArg in,
                      SpinorArg self, SpinorArg out, double c, hipStream_t st) {
  switch (prec) {
    case QXD_F64: return launch_p<QXD_F64>(kind, group, g, f, in, self, out, c, st);
    case QXD_F32: return launch_p<QXD_F32>(kind, group, g, f, in, self, out, c, st);
    case QXD_F16S: return launch_p<QXD_F16S>(kind, group, g, f, in, self, out, c, st);
    case QXD_BF16: return launch_p<QXD_BF16>(kind, group, g, f, in, self, out, c, st);
  }
  return hipErrorInvalidValue;
}

// Autotuned choice of the hop group size, per (precision, kernel kind,
// volume, U(1) phase on the fly): the first call times every candidate on the
// caller's own operands (all candidates compute the same result) and keeps
// the fastest.
struct TuneKey {
  int prec, kind, V, phase;
  bool operator<(const TuneKey &o) const {
    return std::tie(prec, kind, V, phase) < std::tie(o.prec, o.kind, o.V, o.phase);
  }
};
std::mutex g_tune_mu;
std::map<TuneKey, int> g_tuned;

int tune_group(int prec, DiracKind kind, const Geom &g, const OpFields &f, SpinorArg in, SpinorArg self,
               SpinorArg out, double c, hipStream_t st) {
  TuneKey key{prec, (int)kind, g.V, f.qhat != 0};
  {
    std::lock_guard<std::mutex> lk(g_tune_mu);
    auto it = g_tuned.find(key);
    if (it != g_tuned.end()) return it->second;
  }
  static const int cand[] = {1, 2, 4, 8};
  hipEvent_t e0, e1;
  if (hipEventCreate(&e0) != hipSuccess) return 2;
  if (hipEventCreate(&e1) != hipSuccess) {
    (void)hipEventDestroy(e0);
    return 2;
  }
  int best = 2;
  float best_ms = 1e30f;
  for (int gsz : cand) {
    (void)launch_any(prec, kind, gsz, g, f, in, self, out, c, st);  // warm-up
    (void)hipEventRecord(e0, st);
    for (int r = 0; r < 3; r++) (void)launch_any(prec, kind, gsz, g, f, in, self, out, c, st);
    (void)hipEventRecord(e1, st);
    if (hipEventSynchronize(e1) != hipSuccess) break;
    float ms = 0;
    (void)hipEventElapsedTime(&ms, e0, e1);
    if (ms < best_ms) {
      best_ms = ms;
      best = gsz;
    }
  }
  (void)hipEventDestroy(e0);
  (void)hipEventDestroy(e1);
  std::lock_guard<std::mutex> lk(g_tune_mu);
  g_tuned[key] = best;
  return best;
}

}  // namespace

hipError_t launch_dirac(int prec, DiracKind kind, const Geom &g, const OpFields &f, SpinorArg in,
                        SpinorArg self, SpinorArg out, double c, hipStream_t st) {
  if (prec < QXD_F64 || prec > QXD_BF16) return hipErrorInvalidValue;
  int group = kind == DK_PAULI ? 1 : tune_group(prec, kind, g, f, in, self, out, c, st);
  return launch_any(prec, kind, group, g, f, in, self, out, c, st);
}

int tuned_group(int prec, int kind, int V, int phase) {
  std::lock_guard<std::mutex> lk(g_tune_mu);
  auto it = g_tuned.find(TuneKey{prec, kind, V, phase});
  return it == g_tuned.end() ? 0 : it->second;
}

}  // namespace qxd
