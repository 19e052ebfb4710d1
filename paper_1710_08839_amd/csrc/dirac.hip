// Wilson-clover operator kernels: full D, hopping part, Pauli term, and the
// two half-lattice passes of the even-odd Schur complement (Sec. 2.4):
//   odd pass   t_o = D_oo^-1 (self_o + c * acc(in_e))
//   even pass  out_e = P self_e + c * acc(t_o)      (or self_e + c acc)
// so that D^ psi_e = P_e psi_e + acc(t_o)/2 with t_o = -D_oo^-1 acc(psi_e)/2.
// One thread per site; every operand is a structure-of-arrays field in native
// order, so the 64 lanes of a wavefront read consecutive sites.
#include "dirac_site.h"
#include "launch.h"

namespace qxd {

namespace {

template <int P, int KIND>
__global__ void __launch_bounds__(256) dirac_kernel(Geom g, const typename St<P>::pair_t *links,
                                                    const typename St<P>::real_t *angles, int qhat,
                                                    const typename St<P>::pair_t *pauli,
                                                    const typename St<P>::pair_t *pinv,
                                                    Spinor<P> in, Spinor<P> self, Spinor<P> out,
                                                    typename St<P>::comp_t c) {
  using T = typename St<P>::comp_t;
  int t = blockIdx.x * blockDim.x + threadIdx.x;
  int i0 = (KIND == DK_ODD) ? g.Vh : 0;
  int n = (KIND == DK_ODD || KIND == DK_EVEN || KIND == DK_EVEN_ID) ? g.Vh : g.V;
  if (t >= n) return;
  int i = i0 + t;
  cx<T> res[4][3];
  if (KIND != DK_PAULI) {
    Site s = decode(g, i);
    hop_sum<P, T>(g, links, angles, qhat, in, s, i, res);
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

template <int P>
hipError_t launch_p(DiracKind kind, const Geom &g, const OpFields &f, SpinorArg in, SpinorArg self,
                    SpinorArg out, double c, hipStream_t st) {
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
  int n = (kind == DK_ODD || kind == DK_EVEN || kind == DK_EVEN_ID) ? g.Vh : g.V;
  unsigned gr = grid_for(n, 256);
  T cc = (T)c;
  switch (kind) {
    case DK_FULL: dirac_kernel<P, DK_FULL><<<gr, 256, 0, st>>>(g, links, angles, f.qhat, pauli, pinv, vin, vself, vout, cc); break;
    case DK_HOP: dirac_kernel<P, DK_HOP><<<gr, 256, 0, st>>>(g, links, angles, f.qhat, pauli, pinv, vin, vself, vout, cc); break;
    case DK_PAULI: dirac_kernel<P, DK_PAULI><<<gr, 256, 0, st>>>(g, links, angles, f.qhat, pauli, pinv, vin, vself, vout, cc); break;
    case DK_ODD: dirac_kernel<P, DK_ODD><<<gr, 256, 0, st>>>(g, links, angles, f.qhat, pauli, pinv, vin, vself, vout, cc); break;
    case DK_EVEN: dirac_kernel<P, DK_EVEN><<<gr, 256, 0, st>>>(g, links, angles, f.qhat, pauli, pinv, vin, vself, vout, cc); break;
    case DK_EVEN_ID: dirac_kernel<P, DK_EVEN_ID><<<gr, 256, 0, st>>>(g, links, angles, f.qhat, pauli, pinv, vin, vself, vout, cc); break;
  }
  return hipGetLastError();
}

}  // namespace

hipError_t launch_dirac(int prec, DiracKind kind, const Geom &g, const OpFields &f, SpinorArg in,
                        SpinorArg self, SpinorArg out, double c, hipStream_t st) {
  switch (prec) {
    case QXD_F64: return launch_p<QXD_F64>(kind, g, f, in, self, out, c, st);
    case QXD_F32: return launch_p<QXD_F32>(kind, g, f, in, self, out, c, st);
    case QXD_F16S: return launch_p<QXD_F16S>(kind, g, f, in, self, out, c, st);
    case QXD_BF16: return launch_p<QXD_BF16>(kind, g, f, in, self, out, c, st);
  }
  return hipErrorInvalidValue;
}

}  // namespace qxd
