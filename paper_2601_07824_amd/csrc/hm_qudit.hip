// hm_qudit.hip -- pure-state mana of N qudits of odd prime dimension d in {3, 5, 7}.
//
// The qutrit construction of Sec. "Mana for qutrits" holds for every odd prime d (the footnote
// there): with omega = exp(2 pi i / d) and A_0|x> = |-x>, the overlaps <psi|A_ab|psi> for one shift a
// are the Fourier transform over Z_d^N of v_x = conj(alpha_x) alpha_{-x}, alpha = X_a psi
// (alpha_x = psi_{x - a}, digit-wise mod d), with the kernel (F_d)_{jk} = omega^{2jk}
// (Algorithm 4 and Eqs. mana_FT, F3_unnorm_def with 3 -> d).  chi_b(a) is real (A_ab is Hermitian),
// so two shifts a, a + 1 share one complex transform: F(v(a) + i v(a + 1)) = chi(a) + i chi(a + 1).
//
// One workgroup holds the d^N packed values of a shift pair in LDS (at most 157 KB): the product,
// then one pass per digit over the fibres of d values along it (a dense d x d DFT per fibre; a
// thread takes whole fibres, so no barrier is needed inside a stage), then the sums
// sum |chi|, sum chi, sum chi^2 into per-thread FP64 accumulators.  Workgroups take pairs
// blockIdx.x, blockIdx.x + gridDim.x, ...; their FP64 partials are summed in a fixed order.
// The transform is on VALU (complex multiply-adds with the d roots of unity); the state (<= d^N x
// 16 B) is read from L2.
#include <hip/hip_runtime.h>
#include <math.h>
#include <stdint.h>

#include "hm_internal.h"
#include "hm_tile.h"

namespace hm {

namespace {

constexpr uint32_t ipow(uint32_t b, int e) { return e == 0 ? 1u : b * ipow(b, e - 1); }

struct QuditArgs {
  const void *psi;
  int64_t n_pairs;
  double *part;    // [gridDim.x][3]
  double wr[7], wi[7];  // omega^k, k < d
};

// Largest N whose d^N packed values fit one workgroup's LDS (160 KB on gfx950).
template <typename T>
constexpr int qudit_nmax(int d) {
  return sizeof(T) == 4 ? (d == 3 ? 9 : d == 5 ? 6 : 5) : (d == 3 ? 8 : d == 5 ? 5 : 4);
}

template <int D, int N>
struct QuditShape {
  static constexpr uint32_t DN = ipow(D, N);
  static constexpr int NT = DN >= 4096 ? 1024 : DN >= 512 ? 256 : 64;
};

template <typename T, int D, int N>
__global__ __launch_bounds__((QuditShape<D, N>::NT)) void k_qudit_mana(QuditArgs A) {
  constexpr uint32_t DN = QuditShape<D, N>::DN;
  constexpr int NT = QuditShape<D, N>::NT;
  __shared__ vec2<T> v[DN];
  __shared__ double red[3][NT / 64];
  const uint32_t tau = threadIdx.x;
  const vec2<T> *__restrict__ psi = (const vec2<T> *)A.psi;
  T wr[D], wi[D];
#pragma unroll
  for (int k = 0; k < D; ++k) {
    wr[k] = (T)A.wr[k];
    wi[k] = (T)A.wi[k];
  }
  double sm = 0.0, ss = 0.0, sq = 0.0;

  for (int64_t pr = blockIdx.x; pr < A.n_pairs; pr += gridDim.x) {
    const uint32_t a = __builtin_amdgcn_readfirstlane((uint32_t)(2 * pr));
    const bool two = a + 1 < DN;
    // digits of the two shifts (wave-uniform)
    uint32_t ad[N], bd[N];
    {
      uint32_t x = a, y = a + 1;
#pragma unroll
      for (int k = 0; k < N; ++k) {
        ad[k] = x % D;
        bd[k] = y % D;
        x /= D;
        y /= D;
      }
    }
    __syncthreads();  // the previous pair's sums have read v
    for (uint32_t x = tau; x < DN; x += NT) {
      uint32_t i1 = 0, i2 = 0, j1 = 0, j2 = 0, xx = x;
#pragma unroll
      for (int k = 0; k < N; ++k) {
        const uint32_t pw = ipow(D, k);
        const uint32_t xk = xx % D;
        xx /= D;
        // (x - a)_k and (-x - a)_k mod d
        uint32_t t = xk + D - ad[k];
        t = t >= D ? t - D : t;
        uint32_t s = xk + ad[k];
        s = s >= D ? s - D : s;
        s = s == 0 ? 0 : D - s;
        i1 += t * pw;
        i2 += s * pw;
        t = xk + D - bd[k];
        t = t >= D ? t - D : t;
        s = xk + bd[k];
        s = s >= D ? s - D : s;
        s = s == 0 ? 0 : D - s;
        j1 += t * pw;
        j2 += s * pw;
      }
      const vec2<T> p1 = psi[i1], p2 = psi[i2];
      // v(a)_x = conj(alpha_x) alpha_{-x}
      const T vr = p1.x * p2.x + p1.y * p2.y, vi = p1.x * p2.y - p1.y * p2.x;
      T ur = T(0), ui = T(0);
      if (two) {
        const vec2<T> q1 = psi[j1], q2 = psi[j2];
        ur = q1.x * q2.x + q1.y * q2.y;
        ui = q1.x * q2.y - q1.y * q2.x;
      }
      vec2<T> o;
      o.x = vr - ui;  // v(a) + i v(a + 1)
      o.y = vi + ur;
      v[x] = o;
    }
    __syncthreads();
    // one pass per digit k: fibres of d values at stride d^k
#pragma unroll
    for (int k = 0; k < N; ++k) {
      const uint32_t st = ipow(D, k);
      for (uint32_t f = tau; f < DN / D; f += NT) {
        const uint32_t lo = f % st;
        const uint32_t base = (f - lo) * D + lo;
        vec2<T> in[D];
#pragma unroll
        for (int m = 0; m < D; ++m) in[m] = v[base + m * st];
#pragma unroll
        for (int j = 0; j < D; ++j) {
          T yr = in[0].x, yi = in[0].y;
#pragma unroll
          for (int m = 1; m < D; ++m) {
            const int e = (2 * j * m) % D;  // omega^{2jm}
            if (e == 0) {
              yr += in[m].x;
              yi += in[m].y;
            } else {
              yr = fmaT(wr[e], in[m].x, fmaT(-wi[e], in[m].y, yr));
              yi = fmaT(wr[e], in[m].y, fmaT(wi[e], in[m].x, yi));
            }
          }
          vec2<T> o;
          o.x = yr;
          o.y = yi;
          v[base + j * st] = o;
        }
      }
      __syncthreads();
    }
    for (uint32_t b = tau; b < DN; b += NT) {
      const vec2<T> c = v[b];
      const double cr = (double)c.x, ci = two ? (double)c.y : 0.0;
      sm += fabs(cr) + fabs(ci);
      ss += cr + ci;
      sq = fma(cr, cr, fma(ci, ci, sq));
    }
  }
  // fixed-order workgroup sums
  double vals[3] = {sm, ss, sq};
#pragma unroll
  for (int k = 0; k < 3; ++k) {
    double x = vals[k];
    for (int off = 32; off > 0; off >>= 1) x += __shfl_down(x, off, 64);
    if ((tau & 63) == 0) red[k][tau >> 6] = x;
  }
  __syncthreads();
  if (tau == 0) {
    for (int k = 0; k < 3; ++k) {
      double t = 0.0;
      for (int w = 0; w < NT / 64; ++w) t += red[k][w];
      A.part[blockIdx.x * 3 + k] = t;
    }
  }
}

__global__ __launch_bounds__(256) void k_qudit_total(const double *part, int nblk, int n, int d, double *out) {
  __shared__ double red[3][256];
  for (int k = 0; k < 3; ++k) {
    double s = 0.0;
    for (int i = threadIdx.x; i < nblk; i += 256) s += part[i * 3 + k];
    red[k][threadIdx.x] = s;
  }
  __syncthreads();
  for (unsigned w = 128; w > 0; w >>= 1) {
    if (threadIdx.x < w)
      for (int k = 0; k < 3; ++k) red[k][threadIdx.x] += red[k][threadIdx.x + w];
    __syncthreads();
  }
  if (threadIdx.x == 0) {
    const double Dn = pow((double)d, (double)n);
    out[0] = log2(red[0][0] / Dn);  // Eq. mana2 with 3 -> d
    out[1] = red[1][0] / Dn;        // sum_u W(u)
    out[2] = red[2][0] / Dn;        // d^N sum_u W(u)^2
  }
}

// Workgroups: as many as fit the 256 CUs at once (LDS and thread slots), at most one per pair; a
// function of (T, d, N) only, so the partials and their fixed-order sum are reproducible.
template <typename T, int D, int N>
int64_t qudit_grid() {
  constexpr uint32_t DN = QuditShape<D, N>::DN;
  constexpr int NT = QuditShape<D, N>::NT;
  constexpr size_t lds = (size_t)DN * sizeof(vec2<T>) + 3 * (NT / 64) * sizeof(double);
  constexpr int by_lds = (int)((160u * 1024u) / lds), by_thr = 2048 / NT;
  constexpr int per_cu = by_lds < by_thr ? (by_lds < 1 ? 1 : by_lds) : by_thr;
  const int64_t pairs = (DN + 1) / 2, cap = 256 * (int64_t)per_cu;
  return pairs < cap ? pairs : cap;
}

template <typename T, int D, int N>
int launch_n(const void *psi, double *out, void *ws, hipStream_t st) {
  constexpr uint32_t DN = QuditShape<D, N>::DN;
  QuditArgs A{};
  A.psi = psi;
  A.n_pairs = (DN + 1) / 2;
  A.part = (double *)ws;
  for (int k = 0; k < D; ++k) {
    A.wr[k] = cos(2.0 * M_PI * k / D);
    A.wi[k] = sin(2.0 * M_PI * k / D);
  }
  const int64_t grid = qudit_grid<T, D, N>();
  constexpr int nt = QuditShape<D, N>::NT;
  {
    ProfScope prof("mana_qudit", st);
    hipLaunchKernelGGL((k_qudit_mana<T, D, N>), dim3((unsigned)grid), dim3(nt), 0, st, A);
  }
  hipLaunchKernelGGL(k_qudit_total, dim3(1), dim3(256), 0, st, (const double *)A.part, (int)grid, N, D, out);
  return hipPeekAtLastError() == hipSuccess ? OK : fail(E_HIP, "qudit mana launch: %s", hipGetErrorString(hipGetLastError()));
}

template <typename T, int D, int N = 1>
int dispatch(int n, const void *psi, double *out, void *ws, hipStream_t st) {
  if constexpr (N > qudit_nmax<T>(D)) {
    return fail(E_SIZE, "qudit mana: n = %d too large", n);
  } else {
    if (n == N) return launch_n<T, D, N>(psi, out, ws, st);
    return dispatch<T, D, N + 1>(n, psi, out, ws, st);
  }
}

}  // namespace

static constexpr size_t QUDIT_MAX_GRID = 256 * 32;  // 256 CUs x at most 32 workgroups of 64 threads

int qudit_nmax_of(int d, int dbl) { return dbl ? qudit_nmax<double>(d) : qudit_nmax<float>(d); }

int qudit_workspace(int N, int d, int dbl, size_t *bytes) {
  if (d != 3 && d != 5 && d != 7) return fail(E_ARG, "qudit mana: d = %d is not 3, 5 or 7", d);
  const int nmax = qudit_nmax_of(d, dbl);
  if (N < 1 || N > nmax) return fail(E_SIZE, "qudit mana: n = %d outside [1, %d] for d = %d", N, nmax, d);
  *bytes = align256(QUDIT_MAX_GRID * 3 * sizeof(double));
  return OK;
}

int qudit_launch(int N, int d, int dbl, const void *psi, double *out, void *ws, hipStream_t st) {
  if (dbl) {
    if (d == 3) return dispatch<double, 3>(N, psi, out, ws, st);
    if (d == 5) return dispatch<double, 5>(N, psi, out, ws, st);
    return dispatch<double, 7>(N, psi, out, ws, st);
  }
  if (d == 3) return dispatch<float, 3>(N, psi, out, ws, st);
  if (d == 5) return dispatch<float, 5>(N, psi, out, ws, st);
  return dispatch<float, 7>(N, psi, out, ws, st);
}

}  // namespace hm
