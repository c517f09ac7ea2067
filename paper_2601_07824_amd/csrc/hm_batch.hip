// hm_batch.hip -- many qubit states of uneven size in one persistent launch (the batched form of
// Algorithm 2 of "Computing quantum magic of state vectors"; one X-shift of one state is one
// independent workgroup-resident transform, Eq. Z_FT_qubits).
//
// Work units are tiles of the workgroup-resident row pass: a tile holds 2^TB folded values, i.e.
// 2^(TB - nf) whole shift vectors of a state with nf = N - 1 folded bits (one shift at the largest
// size).  The units of all states are numbered in order of decreasing N (largest first, so the long
// units start early and the short ones fill the tail) and handed out by one device counter: each
// workgroup of the persistent grid takes the next unit, finds its state by binary search in the
// state table, runs the tile with that state's row shape and writes the per-shift FP64 sums to the
// state's slots.  One workgroup per state then sums its slots in a fixed order and finalises M_q, so
// the results do not depend on which workgroup took which unit.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <vector>

#include "hm_sre_kern.h"

namespace hm {

struct BatchTab {
  const void *psi;
  int32_t nf;         // folded bits = N - 1
  int32_t orig;       // index of the state in the caller's arrays
  int64_t slot_base;  // first per-shift slot of the state
  int64_t unit_base;  // first work unit of the state
};

static constexpr int TAB_CHUNK = 64;
struct TabChunk {
  BatchTab e[TAB_CHUNK];
};

namespace {

__global__ void k_batch_table(TabChunk c, BatchTab *dst, int count) {
  const int i = threadIdx.x;
  if (i < count) dst[i] = c.e[i];
}

struct BatchArgs {
  const BatchTab *tab;
  int n_states;
  int64_t n_units;
  unsigned long long *counter;
  double *shift_sums;  // [slots][nacc]
  int nacc;
  QArgs qa;
};

// Tiles of a state with nf folded bits when a tile holds 2^TB values (at least one).
__host__ __device__ inline int64_t batch_units(int nf, int TB) {
  const int e = 2 * (nf + 1) - 1 - TB;  // 2^(nf+1) shifts / 2^(TB - nf) shifts per tile
  return e <= 0 ? 1 : (int64_t)1 << e;
}

// LDS of the persistent kernel: the tile's staging buffer and the reduction scratch, sized at launch.
extern __shared__ double batch_lds[];

template <typename T, int NT, int RB>
struct BatchShape {
  static constexpr int TB = ilog2c(NT) + RB;
  using Sh = RowShape<T, NT, RB, TB, true>;
  static constexpr size_t TILE_BYTES = (Sh::LDS_BYTES + 7) / 8 * 8;
  static constexpr size_t LDS_BYTES = TILE_BYTES + (NT / 64 + 1) * sizeof(double);
};

// One tile of one state with row shape NL.  A separate (not inlined) function per shape, so that
// each shape gets its own register allocation instead of the union of all of them.
template <typename T, int NT, int RB, int QM, int NL>
__device__ __noinline__ void batch_tile(const void *psi, int nf, double *shift_sums, int nacc, const QArgs &qa,
                                        int64_t t, uint32_t tau) {
  if constexpr (NL >= RB && NL <= ilog2c(NT) + RB) {
    const StateTileArgs A(psi, nf, shift_sums, nacc, t + 1, qa);
    T *lds = (T *)batch_lds;
    double *red = batch_lds + BatchShape<T, NT, RB>::TILE_BYTES / 8;
    rowpass_tiles<T, NT, RB, NL, false, QM, true, StateTileArgs, true>(A, t, 1, lds, red, tau);
  }
}

template <typename T, int NT, int RB, int QM>
__global__ __launch_bounds__(NT) void k_sre_batch_persistent(BatchArgs B) {
  __shared__ unsigned long long unit_s;
  if (threadIdx.x == 0) unit_s = atomicAdd(B.counter, 1ull);
  __syncthreads();
  // The unit is the same for the whole workgroup: it is read into scalar registers, so everything
  // derived from it (state, pointers, shapes) stays uniform.
  auto read_unit = [&]() -> long long {
    const uint32_t lo32 = __builtin_amdgcn_readfirstlane((uint32_t)unit_s);
    const uint32_t hi32 = __builtin_amdgcn_readfirstlane((uint32_t)(unit_s >> 32));
    return (long long)(((uint64_t)hi32 << 32) | lo32);
  };
  long long u = read_unit();
  int cur = -1;                  // state of the previous unit (consecutive units of a workgroup
  long long cur_lo = 0, cur_hi = 0;  // usually belong to the same state: no search then)
  while (u < B.n_units) {  // every wave leaves once the units are handed out
    // ask for the next unit now; its value is needed only after this tile
    unsigned long long nxt = 0;
    if (threadIdx.x == 0) nxt = atomicAdd(B.counter, 1ull);
    if (!(u >= cur_lo && u < cur_hi)) {
      int lo = 0, hi = B.n_states - 1;
      while (lo < hi) {
        const int mid = (lo + hi + 1) >> 1;
        if (B.tab[mid].unit_base <= u) lo = mid;
        else hi = mid - 1;
      }
      cur = lo;
      cur_lo = B.tab[lo].unit_base;
      cur_hi = lo + 1 < B.n_states ? B.tab[lo + 1].unit_base : B.n_units;
    }
    const BatchTab e = B.tab[cur];
    const int64_t t = u - e.unit_base;
    double *ss = B.shift_sums + e.slot_base * B.nacc;
#define HM_BT(nl) \
  case nl: batch_tile<T, NT, RB, QM, nl>(e.psi, e.nf, ss, B.nacc, B.qa, t, threadIdx.x); break;
    switch (e.nf) {
      HM_BT(4) HM_BT(5) HM_BT(6) HM_BT(7) HM_BT(8) HM_BT(9) HM_BT(10) HM_BT(11) HM_BT(12) HM_BT(13) HM_BT(14)
      HM_BT(15)
      default: break;
    }
#undef HM_BT
    __syncthreads();  // every thread is done with unit_s and the tile's LDS
    if (threadIdx.x == 0) unit_s = nxt;
    __syncthreads();
    u = read_unit();
  }
}

// One workgroup per state: fixed-order sum of its per-shift sums, finalised into
// out[orig (nq + 1) ...] = {M_q..., lost_norm}.
__global__ __launch_bounds__(256) void k_batch_totals(const BatchTab *tab, const double *shift_sums, int nacc, QArgs qa,
                                                      double *out) {
  __shared__ double red[256];
  __shared__ double tot[HM_MAX_Q + 1];
  const BatchTab e = tab[blockIdx.x];
  const uint32_t t = threadIdx.x;
  const int N = e.nf + 1;
  const int64_t ns = (int64_t)1 << N;
  const double *base = shift_sums + e.slot_base * nacc;
  for (int k = 0; k < nacc; ++k) {
    double s = 0.0;
    for (int64_t i = t; i < ns; i += 256) s += base[i * nacc + k];
    red[t] = s;
    __syncthreads();
    for (uint32_t w = 128; w > 0; w >>= 1) {
      if (t < w) red[t] += red[t + w];
      __syncthreads();
    }
    if (t == 0) tot[k] = red[0];
    __syncthreads();
  }
  if (t == 0) {
    double *o = out + (size_t)e.orig * (qa.nq + 1);
    const double D = ldexp(1.0, N);
    for (int i = 0; i < qa.nq; ++i) {
      const double q = qa.q[i];
      o[i] = (q == 1.0) ? -tot[1 + i] / D : log2(tot[1 + i] / D) / (1.0 - q);  // Eq. sre; q -> 1 limit
    }
    o[qa.nq] = 1.0 - tot[0] / D;
  }
}

__global__ void k_batch_zero_counter(unsigned long long *c) { *c = 0ull; }

template <typename T, int NT, int RB, int QM>
static int launch_persistent(const BatchArgs &B, hipStream_t st) {
  static int grid[64] = {};
  int dev = 0;
  if (hipGetDevice(&dev) != hipSuccess || dev < 0 || dev >= 64) return fail(E_HIP, "batched: no current device");
  if (!grid[dev]) {
    int cus = 0, per = 0;
    if (hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess || cus <= 0)
      return fail(E_HIP, "batched: device attribute query failed");
    constexpr size_t lds_q = BatchShape<T, NT, RB>::LDS_BYTES;
    if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&per, k_sre_batch_persistent<T, NT, RB, QM>, NT, lds_q) !=
            hipSuccess || per <= 0)
      per = 1;
    grid[dev] = cus * per;
  }
  const int64_t g = B.n_units < grid[dev] ? B.n_units : grid[dev];
  ProfScope prof("sre_batch_persistent", st);
  constexpr size_t lds_bytes = BatchShape<T, NT, RB>::LDS_BYTES;
  hipLaunchKernelGGL((k_sre_batch_persistent<T, NT, RB, QM>), dim3((unsigned)g), dim3(NT), lds_bytes, st, B);
  return OK;
}

}  // namespace

// Tile bits (log2 of folded values per tile) of the persistent kernel for a largest state of nf_max
// folded bits: the tile must hold one whole shift of it.
static int batch_tb(int nf_max, int dbl) {
  const int RB = dbl ? 4 : 5;
  int tb = RB + 8;  // 256 threads
  while (tb < nf_max) ++tb;
  return tb;
}

bool batch_resident_ok(int N, int dbl) {
  const int nf = N - 1, RB = dbl ? 4 : 5;
  return nf >= RB && nf <= (dbl ? 14 : 15);
}

size_t batch_persistent_workspace(const int *ns, const int *sel, int cnt, int nq, int dbl) {
  size_t slots = 0;
  for (int i = 0; i < cnt; ++i) slots += (size_t)1 << ns[sel[i]];
  (void)dbl;
  return align256((size_t)cnt * sizeof(BatchTab)) + 256 + align256(slots * (size_t)(nq + 1) * sizeof(double));
}

// States sel[0..cnt) (indices into psis / ns, all resident-eligible) in one persistent launch.
int batch_persistent_run(int dbl, const void *const *psis, const int *ns, const int *sel, int cnt, const QArgs &qa,
                         double *out, void *ws, hipStream_t st) {
  if (cnt <= 0) return OK;
  std::vector<int> order(sel, sel + cnt);
  std::stable_sort(order.begin(), order.end(), [&](int a, int b) { return ns[a] > ns[b]; });
  const int nf_max = ns[order[0]] - 1;
  const int TB = batch_tb(nf_max, dbl);
  std::vector<BatchTab> tab(cnt);
  int64_t slots = 0, units = 0;
  for (int j = 0; j < cnt; ++j) {
    const int s = order[j];
    tab[j].psi = psis[s];
    tab[j].nf = ns[s] - 1;
    tab[j].orig = s;
    tab[j].slot_base = slots;
    tab[j].unit_base = units;
    slots += (int64_t)1 << ns[s];
    units += batch_units(ns[s] - 1, TB);
  }
  char *w = (char *)ws;
  BatchTab *dtab = (BatchTab *)w;
  w += align256((size_t)cnt * sizeof(BatchTab));
  unsigned long long *counter = (unsigned long long *)w;
  w += 256;
  double *ss = (double *)w;
  for (int j0 = 0; j0 < cnt; j0 += TAB_CHUNK) {
    TabChunk c{};
    const int k = (cnt - j0) < TAB_CHUNK ? (cnt - j0) : TAB_CHUNK;
    for (int i = 0; i < k; ++i) c.e[i] = tab[j0 + i];
    hipLaunchKernelGGL(k_batch_table, dim3(1), dim3(TAB_CHUNK), 0, st, c, dtab + j0, k);
  }
  BatchArgs B{};
  B.tab = dtab;
  B.n_states = cnt;
  B.n_units = units;
  B.counter = counter;
  B.shift_sums = ss;
  B.nacc = qa.nq + 1;
  B.qa = qa;
  const bool q2 = qa.nq == 1 && qa.q[0] == 2.0;
  int e = OK;
  {
    hipLaunchKernelGGL(k_batch_zero_counter, dim3(1), dim3(1), 0, st, counter);
#define HM_BP(T, NT, RB) e = q2 ? launch_persistent<T, NT, RB, 2>(B, st) : launch_persistent<T, NT, RB, 0>(B, st);
    if (!dbl) {
      if (TB <= 13) { HM_BP(float, 256, 5) }
      else if (TB == 14) { HM_BP(float, 512, 5) }
      else { HM_BP(float, 1024, 5) }
    } else {
      if (TB <= 12) { HM_BP(double, 256, 4) }
      else if (TB == 13) { HM_BP(double, 512, 4) }
      else { HM_BP(double, 1024, 4) }
    }
#undef HM_BP
  }
  if (e) return e;
  ProfScope prof("sre_batch_totals", st);
  hipLaunchKernelGGL(k_batch_totals, dim3((unsigned)cnt), dim3(256), 0, st, (const BatchTab *)dtab, (const double *)ss,
                     qa.nq + 1, qa, out);
  return hipPeekAtLastError() == hipSuccess ? OK : fail(E_HIP, "batched launch: %s", hipGetErrorString(hipGetLastError()));
}

}  // namespace hm
