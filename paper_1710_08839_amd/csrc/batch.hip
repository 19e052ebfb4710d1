// Batched Wilson-clover operator: one launch applies D to the active
// right-hand-side slots of a batch, each slot with its own operator (hopping
// links W = U z^qhat per charge, Pauli term per (q, kappa, csw)).  Work-group
// L in XCD-aware order handles lattice block(s) L / nact for slot
// act[L % nact], so the right-hand sides sharing a block, and with it the
// block's links, run next to each other on one XCD.
#include "batch.h"
#include "dirac_site.h"

namespace qxd {

namespace {

template <int P, int G>
__global__ void __launch_bounds__(256) dirac_batch_kernel(Geom g, const DSlot<P> *slots, const int *act,
                                                          int nact, int bpw) {
  using T = typename St<P>::comp_t;
  const int per_block = 2 * g.Vbh;
  int L = xcd_order(blockIdx.x, gridDim.x);
  int wi = L / nact;
  const DSlot<P> &sl = slots[act[L - wi * nact]];
  int blk = wi * bpw + threadIdx.x / per_block;
  if (blk >= g.nblocks) return;
  int r = threadIdx.x % per_block;
  int par = r >= g.Vbh;
  int i = par * g.Vh + blk * g.Vbh + (par ? r - g.Vbh : r);
  Site s = decode(g, i);
  cx<T> res[4][3], v[4][3], pv[4][3];
  hop_sum<P, T, G>(g, sl.links, nullptr, 0, sl.in, s, i, res);
  load_spinor<P, T>(sl.in, i, v);
  pauli_mul<P, T>(sl.pauli, g, i, v, pv);
#pragma unroll
  for (int a = 0; a < 4; a++)
#pragma unroll
    for (int b = 0; b < 3; b++) res[a][b] = pv[a][b] + (T)(-0.5) * res[a][b];
  store_spinor<P, T>(sl.out, i, res);
}

}  // namespace

template <int P>
hipError_t launch_dirac_batch(const Geom &g, const DSlot<P> *slots, const int *act, int nact, int group,
                              hipStream_t st) {
  if (nact < 1) return hipSuccess;
  int per_block = 2 * g.Vbh;
  if (per_block > 256) return hipErrorInvalidValue;
  int bpw = 256 / per_block;
  unsigned nwg = grid_for(g.nblocks, bpw) * (unsigned)nact;
  int threads = bpw * per_block;
  switch (group) {
    case 1: dirac_batch_kernel<P, 1><<<nwg, threads, 0, st>>>(g, slots, act, nact, bpw); break;
    case 4: dirac_batch_kernel<P, 4><<<nwg, threads, 0, st>>>(g, slots, act, nact, bpw); break;
    default: dirac_batch_kernel<P, 2><<<nwg, threads, 0, st>>>(g, slots, act, nact, bpw); break;
  }
  return hipGetLastError();
}

template hipError_t launch_dirac_batch<QXD_F64>(const Geom &, const DSlot<QXD_F64> *, const int *, int, int, hipStream_t);
template hipError_t launch_dirac_batch<QXD_F32>(const Geom &, const DSlot<QXD_F32> *, const int *, int, int, hipStream_t);
template hipError_t launch_dirac_batch<QXD_F16S>(const Geom &, const DSlot<QXD_F16S> *, const int *, int, int, hipStream_t);
template hipError_t launch_dirac_batch<QXD_BF16>(const Geom &, const DSlot<QXD_BF16> *, const int *, int, int, hipStream_t);

}  // namespace qxd
