// kernels_reduce.hip -- statistics of one batch of rollout outputs (Sec. VI):
// counts and P(collision | H0) (eq. (20)), moments of the stopping distance
// (Table I), the collision-risk curve and exact minimum safe headways
// (Sec. VI-C), and margin statistics.
//
// Sums run in a fixed order (each block a fixed slice, a fixed tree inside the
// block, blocks summed in index order), so repeated calls give identical
// bits.  Order statistics are exact: a histogram over 4,096 value bins
// spanning each array's finite range (plus one bin for the censored +inf
// values) finds the bin holding a target's rank; the bin's elements are
// collected and the rank selected among them in LDS (a radix select over an
// order-preserving map of the FP64 bit patterns).  A bin with more than 8,192
// elements falls back to a radix select over the whole array (8 passes of 8
// bits).
#include <hip/hip_runtime.h>

#include <cmath>
#include <cstring>

#include "aeb_runtime.h"

namespace aeb {

namespace {

constexpr int RB = 256;          // threads per reduction block
constexpr int EB = 1024;         // threads per block of the element passes
constexpr int CP = 4;            // elements per thread loaded together
constexpr int MAX_T = AEB_MAX_RISK + AEB_MAX_MARGIN_Q;
constexpr int NVB = 4096;        // value bins of the selection histograms (+1 overflow)
constexpr int CAP = 8192;        // candidates a target's bin may hold for the LDS sort
constexpr int FB = 1024;         // threads of the finalize / bin-search blocks
// block histogram row: distance value bins | margin value bins | risk-grid ranks
constexpr int HG = 2 * (NVB + 1);             // offset of the risk-grid part
constexpr int HW = HG + AEB_MAX_GRID + 1;     // row width

struct Partial {
  long long ncol, nstop, nimp, nhor, nbnd;
  double sum, dmin, dmax, msum, mmin, mmax;
  float vmax;
  float pad;
  double wmax;     // largest importance-sampling weight
  long long wbad;  // weights that are not finite and >= 0
};

// Selection targets: per target the array (0 censored distance, 1 margin)
// and the 0-based rank.  Passed by value.
struct SelIn {
  int count, n_risk;
  int kind[MAX_T];
  unsigned long long rank[MAX_T];
};

// Selection progress: the value bin holding each target's rank and the rank
// inside the bin, the candidates collected, the binning of each array.
struct Sel {
  int fallback, pad;
  int bin[MAX_T];          // -1: answered without candidates
  unsigned rank_in_bin[MAX_T];
  unsigned bin_count[MAX_T];
  double vmin[2], scale[2];
  int wshift[2];  // fixed-point exponents of w and w^2 (importance-sampling sums)
};

// Radix-select state of the fallback path.
struct SelState {
  unsigned long long prefix[MAX_T];
  unsigned long long rank[MAX_T];
  int kind[MAX_T];
  int count;
  int pad;
};

// order-preserving map of binary64 onto uint64
__device__ inline unsigned long long ordered(double d) {
  unsigned long long u = static_cast<unsigned long long>(__double_as_longlong(d));
  return (u >> 63) ? ~u : (u | 0x8000000000000000ull);
}

__device__ inline double unordered(unsigned long long u) {
  u = (u >> 63) ? (u & 0x7fffffffffffffffull) : ~u;
  return __longlong_as_double(static_cast<long long>(u));
}

__device__ inline double censored(const double* dist, const uint8_t* status, long long i) {
  return (status[i] & 3) == AEB_END_STOP ? dist[i] : INFINITY;
}

// value bin: monotone in v; +inf goes to the overflow bin NVB
__device__ inline int value_bin(double v, double vmin, double scale) {
  if (!(v < INFINITY)) return NVB;
  double f = (v - vmin) * scale;
  int b = f > 0.0 ? static_cast<int>(f) : 0;
  return b < NVB ? b : NVB - 1;
}

// number of grid headways strictly below d, H0_j = lo + j * step (j < ng):
// an arithmetic guess corrected with exact comparisons against the same
// expression, so the count is exact
__device__ inline int grid_rank(double d, double lo, double step, double inv_step, int ng) {
  if (!(d > lo)) return 0;
  if (!(d < INFINITY)) return ng;
  double g = (d - lo) * inv_step;
  int j = g < static_cast<double>(ng) ? static_cast<int>(g) : ng;
  // count = first j with H0_j >= d
  while (j > 0 && !(lo + static_cast<double>(j - 1) * step < d)) --j;
  while (j < ng && lo + static_cast<double>(j) * step < d) ++j;
  return j;
}

template <int NT, typename T, typename Op>
__device__ inline T block_reduce(T v, T* sh, Op op) {
  sh[threadIdx.x] = v;
  __syncthreads();
  for (int w = NT / 2; w > 0; w >>= 1) {
    if (static_cast<int>(threadIdx.x) < w) sh[threadIdx.x] = op(sh[threadIdx.x], sh[threadIdx.x + w]);
    __syncthreads();
  }
  T r = sh[0];
  __syncthreads();
  return r;
}

// exclusive scan of one value per thread over a block of NT threads
template <int NT>
__device__ inline unsigned long long block_exscan(unsigned long long v, unsigned long long* sh) {
  sh[threadIdx.x] = v;
  __syncthreads();
  for (int off = 1; off < NT; off <<= 1) {
    unsigned long long t = threadIdx.x >= static_cast<unsigned>(off) ? sh[threadIdx.x - off] : 0ull;
    __syncthreads();
    sh[threadIdx.x] += t;
    __syncthreads();
  }
  unsigned long long r = sh[threadIdx.x] - v;
  __syncthreads();
  return r;
}

// A 64-bit value moved between lanes by a data-parallel-primitives (DPP)
// modifier; lanes without a source lane under the row and bank masks get `id`.
template <int CTRL, int ROW_MASK, int BANK_MASK>
__device__ inline unsigned long long dpp64(unsigned long long v, unsigned long long id) {
  const unsigned lo = static_cast<unsigned>(__builtin_amdgcn_update_dpp(
      static_cast<int>(static_cast<unsigned>(id)), static_cast<int>(static_cast<unsigned>(v)), CTRL,
      ROW_MASK, BANK_MASK, false));
  const unsigned hi = static_cast<unsigned>(__builtin_amdgcn_update_dpp(
      static_cast<int>(static_cast<unsigned>(id >> 32)), static_cast<int>(static_cast<unsigned>(v >> 32)),
      CTRL, ROW_MASK, BANK_MASK, false));
  return (static_cast<unsigned long long>(hi) << 32) | lo;
}

__device__ inline unsigned long long bits64(double v) {
  return static_cast<unsigned long long>(__double_as_longlong(v));
}
__device__ inline unsigned long long bits64(long long v) { return static_cast<unsigned long long>(v); }
__device__ inline double from_bits(unsigned long long u, double) {
  return __longlong_as_double(static_cast<long long>(u));
}
__device__ inline long long from_bits(unsigned long long u, long long) {
  return static_cast<long long>(u);
}

template <int CTRL, int ROW_MASK, int BANK_MASK, typename T>
__device__ inline T dpp(T v, T id) {
  return from_bits(dpp64<CTRL, ROW_MASK, BANK_MASK>(bits64(v), bits64(id)), v);
}

// Reduction of one value per lane over a wavefront (every lane active): an
// inclusive scan by DPP row shifts of 1, 2, 4, 8 lanes inside each row of 16,
// then row broadcasts of lane 15 and lane 31, leaves the total in lane 63,
// which is read back for every lane.  A fixed association order, so repeated
// calls give the same bits; register moves only, no memory round trips.
template <typename T, typename Op>
__device__ inline T wave_reduce(T v, Op op) {
  const T id = Op::template ident<T>();
  v = op(v, dpp<0x111, 0xf, 0xf>(v, id));  // row_shr:1
  v = op(v, dpp<0x112, 0xf, 0xf>(v, id));  // row_shr:2
  v = op(v, dpp<0x114, 0xf, 0xf>(v, id));  // row_shr:4
  v = op(v, dpp<0x118, 0xf, 0xf>(v, id));  // row_shr:8
  v = op(v, dpp<0x142, 0xa, 0xf>(v, id));  // row_bcast:15 into rows 1 and 3
  v = op(v, dpp<0x143, 0xc, 0xf>(v, id));  // row_bcast:31 into rows 2 and 3
  const unsigned long long u = bits64(v);
  const unsigned lo = static_cast<unsigned>(__builtin_amdgcn_readlane(static_cast<int>(static_cast<unsigned>(u)), 63));
  const unsigned hi = static_cast<unsigned>(__builtin_amdgcn_readlane(static_cast<int>(static_cast<unsigned>(u >> 32)), 63));
  return from_bits((static_cast<unsigned long long>(hi) << 32) | lo, v);
}

struct AddOp {
  template <typename T>
  __device__ T operator()(T a, T b) const { return a + b; }
  template <typename T>
  __device__ static T ident() { return T(0); }
};
struct MinOp {
  __device__ double operator()(double a, double b) const { return b < a ? b : a; }
  template <typename T>
  __device__ static T ident() { return INFINITY; }
};
struct MaxOp {
  __device__ double operator()(double a, double b) const { return b > a ? b : a; }
  template <typename T>
  __device__ static T ident() { return -INFINITY; }
};

__global__ void k_zero_u32(unsigned* p, long long n) {
  long long i = static_cast<long long>(blockIdx.x) * blockDim.x + threadIdx.x;
  if (i < n) p[i] = 0u;
}

__device__ inline void combine(Partial& a, const Partial& b) {
  a.ncol += b.ncol;
  a.nstop += b.nstop;
  a.nimp += b.nimp;
  a.nhor += b.nhor;
  a.nbnd += b.nbnd;
  a.sum += b.sum;
  a.dmin = b.dmin < a.dmin ? b.dmin : a.dmin;
  a.dmax = b.dmax > a.dmax ? b.dmax : a.dmax;
  a.msum += b.msum;
  a.mmin = b.mmin < a.mmin ? b.mmin : a.mmin;
  a.mmax = b.mmax > a.mmax ? b.mmax : a.mmax;
  a.vmax = b.vmax > a.vmax ? b.vmax : a.vmax;
  a.wmax = b.wmax > a.wmax ? b.wmax : a.wmax;
  a.wbad += b.wbad;
}

__device__ inline Partial identity_partial() {
  Partial p;
  p.ncol = p.nstop = p.nimp = p.nhor = p.nbnd = 0;
  p.sum = p.msum = 0.0;
  p.dmin = p.mmin = INFINITY;
  p.dmax = p.mmax = -INFINITY;
  p.vmax = 0.0f;
  p.pad = 0.0f;
  p.wmax = 0.0;
  p.wbad = 0;
  return p;
}

// every field reduced over the wavefront by the fixed butterfly
__device__ inline Partial wave_combine(const Partial& a) {
  Partial p;
  p.ncol = wave_reduce(a.ncol, AddOp());
  p.nstop = wave_reduce(a.nstop, AddOp());
  p.nimp = wave_reduce(a.nimp, AddOp());
  p.nhor = wave_reduce(a.nhor, AddOp());
  p.nbnd = wave_reduce(a.nbnd, AddOp());
  p.sum = wave_reduce(a.sum, AddOp());
  p.dmin = wave_reduce(a.dmin, MinOp());
  p.dmax = wave_reduce(a.dmax, MaxOp());
  p.msum = wave_reduce(a.msum, AddOp());
  p.mmin = wave_reduce(a.mmin, MinOp());
  p.mmax = wave_reduce(a.mmax, MaxOp());
  p.vmax = static_cast<float>(wave_reduce(static_cast<double>(a.vmax), MaxOp()));
  p.pad = 0.0f;
  p.wmax = wave_reduce(a.wmax, MaxOp());
  p.wbad = wave_reduce(a.wbad, AddOp());
  return p;
}

// the block's wavefront partials (in LDS) combined by wavefront 0, lane w
// holding wavefront w's partial; every lane of wavefront 0 gets the result
template <int NW>
__device__ inline Partial block_combine(const Partial* wp) {
  const int l = threadIdx.x;
  return wave_combine(l < NW ? wp[l] : identity_partial());
}

__global__ __launch_bounds__(EB) void k_pass1(OutCols o, long long n, long long chunk,
                                              Partial* part) {
  __shared__ Partial wp[EB / 64];
  const long long lo = static_cast<long long>(blockIdx.x) * chunk;
  const long long hi = lo + chunk < n ? lo + chunk : n;
  long long ncol = 0, nstop = 0, nimp = 0, nhor = 0, nbnd = 0, wbad = 0;
  double sum = 0.0, dmin = INFINITY, dmax = -INFINITY, msum = 0.0, mmin = INFINITY,
         mmax = -INFINITY, wmax = 0.0;
  float vmax = 0.0f;
  if (o.weight) {  // importance-sampling weights: their range and validity
    for (long long i = lo + threadIdx.x; i < hi; i += EB) {
      const double w = o.weight[i];
      if (w >= 0.0 && w < INFINITY)
        wmax = w > wmax ? w : wmax;
      else
        ++wbad;
    }
  }
  // CP elements per thread are loaded before any is used (chunk = CP * EB)
  for (long long i0 = lo; i0 < hi; i0 += static_cast<long long>(EB) * CP) {
    uint8_t sv[CP];
    double dv[CP], mv[CP];
    float vv[CP];
#pragma unroll
    for (int p = 0; p < CP; ++p) {
      const long long i = i0 + p * EB + threadIdx.x;
      sv[p] = 0;
      dv[p] = mv[p] = 0.0;
      vv[p] = 0.0f;
      if (i < hi) {
        sv[p] = o.status[i];
        dv[p] = o.dist[i];
        mv[p] = o.margin[i];
        vv[p] = o.vimp[i];
      }
    }
#pragma unroll
    for (int p = 0; p < CP; ++p) {
    if (i0 + p * EB + threadIdx.x >= hi) break;
    const uint8_t st = sv[p];
    if (st & AEB_BOUNDARY) ++nbnd;
    const double d = dv[p];
    const double m = mv[p];
    const int end = st & 3;
    if (st & AEB_COLLIDED) {
      ++ncol;
      const float vi = vv[p];
      vmax = vi > vmax ? vi : vmax;
    }
    if (end == AEB_END_STOP) {
      ++nstop;
      sum += d;
      dmin = d < dmin ? d : dmin;
      dmax = d > dmax ? d : dmax;
    } else if (end == AEB_END_IMPACT) {
      ++nimp;
    } else if (end == AEB_END_HORIZON) {
      ++nhor;
    }
    msum += m;
    mmin = m < mmin ? m : mmin;
    mmax = m > mmax ? m : mmax;
    }
  }
  // wavefront partials, then the block's waves combined in index order
  Partial p;
  p.ncol = ncol;
  p.nstop = nstop;
  p.nimp = nimp;
  p.nhor = nhor;
  p.nbnd = nbnd;
  p.sum = sum;
  p.dmin = dmin;
  p.dmax = dmax;
  p.msum = msum;
  p.mmin = mmin;
  p.mmax = mmax;
  p.vmax = vmax;
  p.pad = 0.0f;
  p.wmax = wmax;
  p.wbad = wbad;
  p = wave_combine(p);
  if ((threadIdx.x & 63) == 0) wp[threadIdx.x >> 6] = p;
  __syncthreads();
  if (threadIdx.x < 64) {
    const Partial q = block_combine<EB / 64>(wp);
    if (threadIdx.x == 0) part[blockIdx.x] = q;
  }
}

// Combine the block partials in a fixed order (thread t takes partials
// t, t+FB, ... in order, then a fixed tree).
__global__ __launch_bounds__(FB) void k_fin1(const Partial* part, int nb, long long n,
                                             int weighted, aeb_stats* st, Sel* sel) {
  __shared__ Partial wp[FB / 64];
  Partial p = identity_partial();
  for (int b = threadIdx.x; b < nb; b += FB) combine(p, part[b]);
  p = wave_combine(p);
  if ((threadIdx.x & 63) == 0) wp[threadIdx.x >> 6] = p;
  __syncthreads();
  if (threadIdx.x >= 64) return;
  const Partial q = block_combine<FB / 64>(wp);
  const long long ncol = q.ncol, nstop = q.nstop, nimp = q.nimp, nhor = q.nhor, nbnd = q.nbnd;
  const double sum = q.sum, dmin = q.dmin, dmax = q.dmax, msum = q.msum, mmin = q.mmin,
               mmax = q.mmax;
  const double vmax = q.vmax;
  if (threadIdx.x == 0) {
    st->n = n;
    st->n_collide = ncol;
    st->n_stop = nstop;
    st->n_impact = nimp;
    st->n_horizon = nhor;
    st->n_boundary = nbnd;
    st->p_collision = static_cast<double>(ncol) / static_cast<double>(n);
    st->mean_dist = nstop > 0 ? sum / static_cast<double>(nstop) : NAN;
    st->dist_min = nstop > 0 ? dmin : NAN;
    st->dist_max = nstop > 0 ? dmax : NAN;
    st->sd_dist = NAN;
    st->margin_min = mmin;
    st->margin_mean = msum / static_cast<double>(n);
    st->v_impact_max = static_cast<float>(vmax);
    // value bins span the finite range of each selected array
    sel->vmin[0] = nstop > 0 ? dmin : 0.0;
    sel->scale[0] = (nstop > 0 && dmax > dmin) ? static_cast<double>(NVB) / (dmax - dmin) : 0.0;
    sel->vmin[1] = mmin;
    sel->scale[1] = mmax > mmin ? static_cast<double>(NVB) / (mmax - mmin) : 0.0;
    // fixed point of the weighted sums: value * 2^shift as a 128-bit integer,
    // with n * max value * 2^shift < 2^126 (no sum can overflow)
    int ln = 0;
    while ((1ll << ln) < n) ++ln;
    int e1 = 0, e2 = 0;
    frexp(q.wmax, &e1);
    frexp(q.wmax * q.wmax, &e2);
    sel->wshift[0] = q.wmax > 0.0 ? 126 - ln - e1 : 0;
    sel->wshift[1] = q.wmax > 0.0 ? 126 - ln - e2 : 0;
    st->weighted = weighted ? (q.wbad > 0 ? -1 : 1) : 0;
  }
}

// Sum of squared deviations for the sd, and block-private histograms (LDS,
// written out without atomics): value bins of the arrays that have targets,
// and the number of risk-grid headways below each censored distance.
__global__ __launch_bounds__(EB) void k_pass2(OutCols o, long long n, long long chunk,
                                              const aeb_stats* st, const Sel* sel, int need_d,
                                              int need_m, double glo, double gstep,
                                              double ginv, int ng,
                                              int hw, unsigned* bhist, double* part) {
  __shared__ double shd[EB / 64];
  __shared__ unsigned h[HW];
  for (int j = threadIdx.x; j < hw; j += EB) h[j] = 0;
  __syncthreads();
  const double mean = st->mean_dist;
  const double vmin0 = sel->vmin[0], sc0 = sel->scale[0];
  const double vmin1 = sel->vmin[1], sc1 = sel->scale[1];
  const long long lo = static_cast<long long>(blockIdx.x) * chunk;
  const long long hi = lo + chunk < n ? lo + chunk : n;
  double ss = 0.0;
  // CP elements per thread are loaded before any is used (chunk2 = CP * EB)
  for (long long i0 = lo; i0 < hi; i0 += static_cast<long long>(EB) * CP) {
    uint8_t sv[CP];
    double dv[CP], mv[CP];
#pragma unroll
    for (int p = 0; p < CP; ++p) {
      const long long i = i0 + p * EB + threadIdx.x;
      sv[p] = 0;
      dv[p] = mv[p] = 0.0;
      if (i < hi) {
        sv[p] = o.status[i];
        dv[p] = o.dist[i];
        mv[p] = o.margin[i];
      }
    }
#pragma unroll
    for (int p = 0; p < CP; ++p) {
      if (i0 + p * EB + threadIdx.x >= hi) break;
      const bool stop = (sv[p] & 3) == AEB_END_STOP;
      const double d = dv[p];
      if (stop) {
        const double e = d - mean;
        ss += e * e;
      }
      if (need_d) atomicAdd(&h[value_bin(stop ? d : INFINITY, vmin0, sc0)], 1u);
      if (need_m) atomicAdd(&h[(NVB + 1) + value_bin(mv[p], vmin1, sc1)], 1u);
      if (ng >= 2) atomicAdd(&h[HG + grid_rank(stop ? d : INFINITY, glo, gstep, ginv, ng)], 1u);
    }
  }
  ss = wave_reduce(ss, AddOp());
  if ((threadIdx.x & 63) == 0) shd[threadIdx.x >> 6] = ss;
  __syncthreads();
  if (threadIdx.x == 0) {
    double t = shd[0];
    for (int w = 1; w < EB / 64; ++w) t += shd[w];
    part[blockIdx.x] = t;
  }
  unsigned* out = bhist + static_cast<size_t>(blockIdx.x) * hw;
  for (int j = threadIdx.x; j < hw; j += EB) out[j] = h[j];
}

// ---- importance-sampling sums: exact 128-bit fixed point ----
// A nonnegative value as the integer floor(value * 2^shift) in two words
// (the scaling by a power of two and the split are exact in binary64).
__device__ inline void to_fixed(double v, int shift, unsigned long long& hi,
                                unsigned long long& lo) {
  const double t = ldexp(v, shift);
  const double h = floor(ldexp(t, -64));
  hi = static_cast<unsigned long long>(h);
  lo = static_cast<unsigned long long>(t - ldexp(h, 64));
}

// acc[0] low word, acc[1] high word; integer adds in any order give the
// same total, so the sums do not depend on scheduling
__device__ inline void add_fixed(unsigned long long* acc, unsigned long long hi,
                                 unsigned long long lo) {
  if (lo) {
    const unsigned long long old = atomicAdd(&acc[0], lo);
    if (old + lo < old) atomicAdd(&acc[1], 1ull);
  }
  if (hi) atomicAdd(&acc[1], hi);
}

__device__ inline double from_fixed(unsigned long long hi, unsigned long long lo, int shift) {
  return ldexp(static_cast<double>(hi), 64 - shift) + ldexp(static_cast<double>(lo), -shift);
}

// Per block (the histogram pass's slices): for each risk-grid rank bin the
// sums of w and w^2, then bins for the collided samples and for all samples;
// four words per bin (w low, w high, w^2 low, w^2 high), merged into the
// zeroed global accumulators.
constexpr int WACC = (AEB_MAX_GRID + 3) * 4;
__global__ __launch_bounds__(EB) void k_wpass(OutCols o, long long n, long long chunk, double glo,
                                              double gstep, double ginv, int ng, const Sel* sel,
                                              unsigned long long* gacc) {
  __shared__ unsigned long long acc[WACC];
  const int G = ng >= 2 ? ng + 1 : 0;  // rank bins 0..ng
  const int nacc = (G + 2) * 4;
  for (int j = threadIdx.x; j < nacc; j += EB) acc[j] = 0ull;
  __syncthreads();
  const int s1 = sel->wshift[0], s2 = sel->wshift[1];
  const long long lo = static_cast<long long>(blockIdx.x) * chunk;
  const long long hi = lo + chunk < n ? lo + chunk : n;
  for (long long i = lo + threadIdx.x; i < hi; i += EB) {
    const double w = o.weight[i];
    if (!(w >= 0.0 && w < INFINITY)) continue;  // reported through the statistics' flag
    const uint8_t st = o.status[i];
    const double d = o.dist[i];
    unsigned long long h1, l1, h2, l2;
    to_fixed(w, s1, h1, l1);
    to_fixed(w * w, s2, h2, l2);
    if (G) {
      const int b = grid_rank((st & 3) == AEB_END_STOP ? d : INFINITY, glo, gstep, ginv, ng);
      add_fixed(&acc[4 * b], h1, l1);
      add_fixed(&acc[4 * b + 2], h2, l2);
    }
    if (st & AEB_COLLIDED) {
      add_fixed(&acc[4 * G], h1, l1);
      add_fixed(&acc[4 * G + 2], h2, l2);
    }
    add_fixed(&acc[4 * (G + 1)], h1, l1);
  }
  __syncthreads();
  for (int j = threadIdx.x; j < nacc / 2; j += EB) {
    const unsigned long long l = acc[2 * j], h = acc[2 * j + 1];
    if (l | h) add_fixed(&gacc[2 * j], h, l);
  }
}

// The weighted estimates from the accumulated sums (one thread, in a fixed
// order): suffix sums over the rank bins from the top give sum w [D > H0_j].
__global__ void k_wfin(long long n, int ng, const Sel* sel, const unsigned long long* gacc,
                       aeb_stats* st) {
  if (threadIdx.x != 0) return;
  const int G = ng >= 2 ? ng + 1 : 0;
  const double nd = static_cast<double>(n);
  const int s1 = sel->wshift[0], s2 = sel->wshift[1];
  if (st->weighted != 1) {
    st->p_collision_w = st->p_collision_se = st->weight_mean = NAN;
    for (int j = 0; j < ng; ++j) st->risk_pw[j] = st->risk_se[j] = NAN;
    return;
  }
  auto se_of = [&](double p, double m2) {
    const double v = m2 / nd - p * p;
    return n > 1 ? sqrt((v > 0.0 ? v : 0.0) / (nd - 1.0)) : NAN;
  };
  unsigned long long a_l = 0, a_h = 0, b_l = 0, b_h = 0;  // suffix sums of w and w^2
  for (int b = G - 1; b >= 1; --b) {
    const unsigned long long* c = gacc + 4 * b;
    const unsigned long long al = a_l + c[0];
    a_h += c[1] + (al < a_l ? 1ull : 0ull);
    a_l = al;
    const unsigned long long bl = b_l + c[2];
    b_h += c[3] + (bl < b_l ? 1ull : 0ull);
    b_l = bl;
    const double p = from_fixed(a_h, a_l, s1) / nd;
    st->risk_pw[b - 1] = p;
    st->risk_se[b - 1] = se_of(p, from_fixed(b_h, b_l, s2));
  }
  const unsigned long long* c = gacc + 4 * G;
  const double pc = from_fixed(c[1], c[0], s1) / nd;
  st->p_collision_w = pc;
  st->p_collision_se = se_of(pc, from_fixed(c[3], c[2], s2));
  st->weight_mean = from_fixed(gacc[4 * (G + 1) + 1], gacc[4 * (G + 1)], s1) / nd;
}

// Bin totals of the block-private histograms: a 2-D grid, each thread sums
// BT_ROWS blocks' counts of one bin (adjacent threads, adjacent bins) and adds
// them to the zeroed totals (integer adds: order-free).
constexpr int BT_ROWS = 16;
__global__ __launch_bounds__(256) void k_bin_totals(const unsigned* bhist, int nb, int hw,
                                                    unsigned* btot) {
  const int j = blockIdx.x * 256 + threadIdx.x;
  if (j >= hw) return;
  const int b0 = blockIdx.y * BT_ROWS;
  const int b1 = b0 + BT_ROWS < nb ? b0 + BT_ROWS : nb;
  unsigned c = 0;
  for (int b = b0; b < b1; ++b) c += bhist[static_cast<size_t>(b) * hw + j];
  if (c) atomicAdd(&btot[j], c);
}

// Block 0: the sd and the risk curve.  Block 1 + t: find the value bin
// holding target t's rank.
__global__ __launch_bounds__(FB) void k_fin2(const double* part, int nb, long long n, int ng,
                                             aeb_stats* st, Sel* sel, SelIn in,
                                             const unsigned* btot, const unsigned* bhist, int hw,
                                             unsigned* boff) {
  __shared__ double shd[FB];
  __shared__ unsigned long long shu[FB];
  __shared__ int s_bin;
  if (blockIdx.x == 0) {
    double ss = 0.0;
    for (int b = threadIdx.x; b < nb; b += FB) ss += part[b];
    ss = block_reduce<FB>(ss, shd, AddOp());
    if (threadIdx.x == 0)
      st->sd_dist = st->n_stop > 1 ? sqrt(ss / static_cast<double>(st->n_stop - 1)) : NAN;
    // risk curve: #{D > H0_j} = n - #{D with at most j headways below it}
    const unsigned* gh = btot + HG;
    constexpr int PER = (AEB_MAX_GRID + FB - 1) / FB;
    unsigned long long loc = 0;
    for (int q = 0; q < PER; ++q) {
      const int j = threadIdx.x * PER + q;
      if (j < ng) loc += gh[j];
    }
    unsigned long long before = block_exscan<FB>(loc, shu);
    for (int q = 0; q < PER; ++q) {
      const int j = threadIdx.x * PER + q;
      if (j < ng) {
        before += gh[j];
        const long long above = n - static_cast<long long>(before);
        st->risk_count[j] = above;
        st->risk_p[j] = static_cast<double>(above) / static_cast<double>(n);
      }
    }
    return;
  }
  const int t = blockIdx.x - 1;
  if (t >= in.count) return;
  if (threadIdx.x == 0) s_bin = -1;
  const unsigned* tot = btot + (in.kind[t] ? (NVB + 1) : 0);
  constexpr int PER = (NVB + 1 + FB - 1) / FB;
  unsigned cnt[PER];
  unsigned long long loc = 0;
  for (int q = 0; q < PER; ++q) {
    const int j = threadIdx.x * PER + q;
    cnt[q] = j <= NVB ? tot[j] : 0u;
    loc += cnt[q];
  }
  const unsigned long long r = in.rank[t];
  unsigned long long before = block_exscan<FB>(loc, shu);
  if (r >= before && r < before + loc) {
    for (int q = 0; q < PER; ++q) {
      const int j = threadIdx.x * PER + q;
      if (j > NVB) break;
      if (r < before + cnt[q]) {
        sel->rank_in_bin[t] = static_cast<unsigned>(r - before);
        sel->bin_count[t] = cnt[q];
        if (j == NVB) {  // the rank falls among the censored (+inf) samples
          sel->bin[t] = -1;
          if (t < in.n_risk) st->headway[t] = INFINITY;
        } else if (cnt[q] > CAP) {
          sel->bin[t] = -1;
          atomicOr(&sel->fallback, 1);
        } else {
          sel->bin[t] = j;
          s_bin = j;
        }
        break;
      }
      before += cnt[q];
    }
  }
  __syncthreads();
  // where each histogram block's elements of the bin go among the candidates:
  // an exclusive scan of the block histograms' counts of that bin, so the
  // collection needs no global atomics (it uses the histogram pass's blocks)
  const int j = s_bin;
  if (j < 0) return;
  const int col = (in.kind[t] ? (NVB + 1) : 0) + j;
  unsigned long long carry = 0;
  for (int b0 = 0; b0 < nb; b0 += FB) {
    const int b = b0 + static_cast<int>(threadIdx.x);
    const unsigned long long c = b < nb ? bhist[static_cast<size_t>(b) * hw + col] : 0ull;
    const unsigned long long ex = block_exscan<FB>(c, shu);
    if (b < nb) boff[static_cast<size_t>(t) * nb + b] = static_cast<unsigned>(carry + ex);
    if (threadIdx.x == FB - 1) shu[0] = ex + c;  // the tile's total
    __syncthreads();
    carry += shu[0];
    __syncthreads();
  }
}

// Collect the keys of every element in a target's bin: block b of the
// histogram pass's decomposition writes its elements from the offset the bin
// search computed for it, ranked inside the block by LDS counters.
__global__ __launch_bounds__(EB) void k_collect(OutCols o, long long n, long long chunk, Sel* sel,
                                                SelIn in, const unsigned* boff,
                                                unsigned long long* cand) {
  __shared__ int tb[MAX_T], tk[MAX_T];
  __shared__ unsigned lc[MAX_T], lbase[MAX_T];
  __shared__ double vmin[2], scale[2];
  const int T = in.count;
  if (static_cast<int>(threadIdx.x) < T) {
    tb[threadIdx.x] = sel->bin[threadIdx.x];
    tk[threadIdx.x] = in.kind[threadIdx.x];
    lc[threadIdx.x] = 0u;
    lbase[threadIdx.x] =
        tb[threadIdx.x] >= 0 ? boff[static_cast<size_t>(threadIdx.x) * gridDim.x + blockIdx.x] : 0u;
  }
  if (threadIdx.x < 2) {
    vmin[threadIdx.x] = sel->vmin[threadIdx.x];
    scale[threadIdx.x] = sel->scale[threadIdx.x];
  }
  __syncthreads();
  const long long lo = static_cast<long long>(blockIdx.x) * chunk;
  const long long hi = lo + chunk < n ? lo + chunk : n;
  // each pass loads CP elements per thread before using any of them
  for (long long i0 = lo; i0 < hi; i0 += static_cast<long long>(EB) * CP) {
    uint8_t stt[CP];
    double dv[CP], mv[CP];
#pragma unroll
    for (int p = 0; p < CP; ++p) {
      const long long i = i0 + p * EB + threadIdx.x;
      stt[p] = 0;
      dv[p] = mv[p] = 0.0;
      if (i < hi) {
        stt[p] = o.status[i];
        dv[p] = o.dist[i];
        mv[p] = o.margin[i];
      }
    }
#pragma unroll
    for (int p = 0; p < CP; ++p) {
      const bool ok = i0 + p * EB + threadIdx.x < hi;
      const double dc = (stt[p] & 3) == AEB_END_STOP ? dv[p] : INFINITY;
      const double m = mv[p];
      const int bd = value_bin(dc, vmin[0], scale[0]);
      const int bm = value_bin(m, vmin[1], scale[1]);
      // most wavefronts hold no element of any target's bin: one test first
      bool any = false;
#pragma unroll
      for (int t = 0; t < MAX_T; ++t)
        if (t < T) any = any || (tb[t] >= 0 && (tk[t] ? bm : bd) == tb[t]);
      if (!(ok && any)) continue;
      for (int t = 0; t < T; ++t) {
        const int b = tk[t] ? bm : bd;
        if (tb[t] >= 0 && b == tb[t]) {
          const unsigned slot = lbase[t] + atomicAdd(&lc[t], 1u);
          if (slot < CAP) cand[t * CAP + slot] = ordered(tk[t] ? m : dc);
        }
      }
    }
  }
}

// One block per target: the element of rank r among the bin's candidates by
// a most-significant-digit radix select in LDS, starting at the first byte
// in which the candidates differ (they share the bin's leading bits).
__global__ __launch_bounds__(RB) void k_pick(const Sel* sel, SelIn in,
                                             const unsigned long long* cand, aeb_stats* st) {
  __shared__ unsigned long long key[CAP];
  __shared__ unsigned hist[256];
  __shared__ unsigned long long wlo[RB / 64], whi[RB / 64];
  __shared__ unsigned long long s_prefix;
  __shared__ unsigned s_rank;
  const int t = blockIdx.x;
  // the host reads the fallback flag through the statistics' reserved word
  if (t == 0 && threadIdx.x == 0) st->reserved = sel->fallback;
  if (t >= in.count || sel->bin[t] < 0) return;
  // every element of the bin was collected (the bin holds at most CAP)
  const unsigned m = sel->bin_count[t] < CAP ? sel->bin_count[t] : CAP;
  unsigned long long lo = ~0ull, hi = 0ull;
  for (unsigned j = threadIdx.x; j < m; j += RB) {
    const unsigned long long k = cand[t * CAP + j];
    key[j] = k;
    lo = k < lo ? k : lo;
    hi = k > hi ? k : hi;
  }
  for (int o = 32; o > 0; o >>= 1) {
    const unsigned long long a = __shfl_xor(lo, o), b = __shfl_xor(hi, o);
    lo = a < lo ? a : lo;
    hi = b > hi ? b : hi;
  }
  if ((threadIdx.x & 63) == 0) {
    wlo[threadIdx.x >> 6] = lo;
    whi[threadIdx.x >> 6] = hi;
  }
  __syncthreads();
  lo = wlo[0];
  hi = whi[0];
  for (int w = 1; w < RB / 64; ++w) {
    lo = wlo[w] < lo ? wlo[w] : lo;
    hi = whi[w] > hi ? whi[w] : hi;
  }
  const unsigned long long diff = lo ^ hi;
  const int first = diff ? __clzll(static_cast<long long>(diff)) / 8 : 8;  // first differing byte
  if (threadIdx.x == 0) {
    s_prefix = first == 0 ? 0ull : (lo & (~0ull << (64 - 8 * first)));
    s_rank = sel->rank_in_bin[t];
  }
  __syncthreads();
  for (int pass = first; pass < 8; ++pass) {
    const int shift = 56 - 8 * pass;
    const unsigned long long mask = pass == 0 ? 0ull : (~0ull << (64 - 8 * pass));
    const unsigned long long pre = s_prefix;
    hist[threadIdx.x] = 0;  // RB == 256 bins
    __syncthreads();
    for (unsigned j = threadIdx.x; j < m; j += RB) {
      const unsigned long long k = key[j];
      if ((k & mask) == pre) atomicAdd(&hist[(k >> shift) & 255ull], 1u);
    }
    __syncthreads();
    if (threadIdx.x < 64) {
      // wave 0: digit whose cumulative count passes the rank (4 bins per lane)
      const int l = threadIdx.x;
      unsigned c[4], tot = 0;
      for (int q = 0; q < 4; ++q) {
        c[q] = hist[4 * l + q];
        tot += c[q];
      }
      unsigned inc = tot;  // inclusive scan over lanes
      for (int o = 1; o < 64; o <<= 1) {
        const unsigned v = __shfl_up(inc, o);
        if (l >= o) inc += v;
      }
      const unsigned r = s_rank;
      unsigned before = inc - tot;
      if (r >= before && r < inc) {
        for (int q = 0; q < 4; ++q) {
          if (r < before + c[q]) {
            s_prefix = pre | (static_cast<unsigned long long>(4 * l + q) << shift);
            s_rank = r - before;
            break;
          }
          before += c[q];
        }
      }
    }
    __syncthreads();
  }
  if (threadIdx.x == 0) {
    const double v = unordered(first == 8 ? lo : s_prefix);
    if (t < in.n_risk)
      st->headway[t] = v;
    else
      st->margin_q[t - in.n_risk] = v;
  }
}

// ---- fallback: most-significant-digit radix select, 8 passes of 8 bits ----
__global__ __launch_bounds__(RB) void k_select_hist(OutCols o, long long n, long long chunk,
                                                    const SelState* ss, int pass, unsigned* ghist) {
  __shared__ unsigned hist[MAX_T * 256];
  __shared__ unsigned long long pre[MAX_T];
  __shared__ int kind[MAX_T];
  const int T = ss->count;
  for (int j = threadIdx.x; j < T * 256; j += RB) hist[j] = 0;
  if (static_cast<int>(threadIdx.x) < T) {
    pre[threadIdx.x] = ss->prefix[threadIdx.x];
    kind[threadIdx.x] = ss->kind[threadIdx.x];
  }
  __syncthreads();
  const int shift = 56 - 8 * pass;
  const unsigned long long mask = pass == 0 ? 0ull : (~0ull << (64 - 8 * pass));
  const long long lo = static_cast<long long>(blockIdx.x) * chunk;
  const long long hi = lo + chunk < n ? lo + chunk : n;
  for (long long i = lo + threadIdx.x; i < hi; i += RB) {
    const unsigned long long kd = ordered(censored(o.dist, o.status, i));
    const unsigned long long km = ordered(o.margin[i]);
    for (int t = 0; t < T; ++t) {
      const unsigned long long key = kind[t] ? km : kd;
      if ((key & mask) == (pre[t] & mask))
        atomicAdd(&hist[t * 256 + static_cast<int>((key >> shift) & 255ull)], 1u);
    }
  }
  __syncthreads();
  for (int j = threadIdx.x; j < T * 256; j += RB)
    if (hist[j]) atomicAdd(&ghist[j], hist[j]);
}

__global__ void k_select_step(SelState* ss, int pass, unsigned* ghist) {
  const int t = threadIdx.x;
  if (t >= ss->count) return;
  unsigned* h = ghist + t * 256;
  unsigned long long r = ss->rank[t];
  int d = 0;
  for (; d < 255; ++d) {
    if (r < h[d]) break;
    r -= h[d];
  }
  ss->rank[t] = r;
  ss->prefix[t] |= static_cast<unsigned long long>(d) << (56 - 8 * pass);
  for (int j = 0; j < 256; ++j) h[j] = 0;
}

__global__ void k_select_out(const SelState* ss, int n_risk, aeb_stats* st) {
  const int t = threadIdx.x;
  if (t >= ss->count) return;
  const double v = unordered(ss->prefix[t]);
  if (t < n_risk)
    st->headway[t] = v;
  else
    st->margin_q[t - n_risk] = v;
}

size_t align256(size_t b) { return (b + 255) & ~size_t(255); }

}  // namespace

namespace {

// Scratch layout of one reduction: stats, selection state and the bin totals
// (selection bins and risk-grid ranks) first (zeroed by one launch), then the
// block partials, the block histograms, the candidates and the radix-select
// state.
struct RLayout {
  long long chunk, chunk2;
  int nb, nb2, T;
  size_t off_sel, off_zero_end, off_var, off_bh, off_bt, off_wa, off_bo, off_cand, off_ss, off_sh,
      total;
};

RLayout layout(int64_t n, const aeb_reduce_req& req) {
  RLayout L;
  // element passes: 4,096 elements per block of 1,024 threads (measured faster
  // than smaller blocks or slices: fewer partials, block histograms and
  // per-block fixed costs)
  L.chunk = EB * CP;
  L.chunk2 = EB * CP;
  L.nb = static_cast<int>((n + L.chunk - 1) / L.chunk);
  L.nb2 = static_cast<int>((n + L.chunk2 - 1) / L.chunk2);
  L.T = req.n_risk + req.n_margin_q;
  const int tc = L.T > 0 ? L.T : 1;
  L.off_sel = align256(sizeof(aeb_stats));
  L.off_bt = align256(L.off_sel + sizeof(Sel));
  L.off_wa = align256(L.off_bt + sizeof(unsigned) * HW);
  L.off_zero_end = align256(L.off_wa + sizeof(unsigned long long) * WACC);
  L.off_var = align256(L.off_zero_end + sizeof(Partial) * L.nb);
  L.off_bh = align256(L.off_var + sizeof(double) * (L.nb > L.nb2 ? L.nb : L.nb2));
  L.off_bo = align256(L.off_bh + sizeof(unsigned) * HW * L.nb2);
  L.off_cand = align256(L.off_bo + sizeof(unsigned) * tc * L.nb2);
  L.off_ss = align256(L.off_cand + sizeof(unsigned long long) * tc * CAP);
  L.off_sh = align256(L.off_ss + sizeof(SelState));
  L.total = align256(L.off_sh + sizeof(unsigned) * tc * 256);
  return L;
}

}  // namespace

size_t reduce_scratch_bytes(int64_t n, const aeb_reduce_req& req) { return layout(n, req).total; }

int reduce_enqueue(const OutCols& out, int64_t n, const aeb_reduce_req& req, void* scratch_base,
                   aeb_stats* host_out, hipStream_t st) {
  const RLayout L = layout(n, req);
  const int ng = req.n_grid;
  const int T = L.T;
  char* base = static_cast<char*>(scratch_base);
  aeb_stats* dstats = reinterpret_cast<aeb_stats*>(base);
  Sel* sel = reinterpret_cast<Sel*>(base + L.off_sel);
  Partial* part = reinterpret_cast<Partial*>(base + L.off_zero_end);
  double* vpart = reinterpret_cast<double*>(base + L.off_var);
  unsigned* bhist = reinterpret_cast<unsigned*>(base + L.off_bh);
  unsigned* btot = reinterpret_cast<unsigned*>(base + L.off_bt);
  unsigned* boff = reinterpret_cast<unsigned*>(base + L.off_bo);
  unsigned long long* wacc = reinterpret_cast<unsigned long long*>(base + L.off_wa);
  unsigned long long* cand = reinterpret_cast<unsigned long long*>(base + L.off_cand);

  // targets: ranks computed exactly as floor(level * N) in binary64
  SelIn in;
  std::memset(&in, 0, sizeof(in));
  in.count = T;
  in.n_risk = req.n_risk;
  bool need_d = false, need_m = false;
  for (int j = 0; j < req.n_risk; ++j) {
    long long m = static_cast<long long>(std::floor(req.risk[j] * static_cast<double>(n)));
    in.rank[j] = static_cast<unsigned long long>(n - m - 1);
    in.kind[j] = 0;
    need_d = true;
  }
  for (int j = 0; j < req.n_margin_q; ++j) {
    long long m = static_cast<long long>(std::floor(req.margin_q[j] * static_cast<double>(n)));
    in.rank[req.n_risk + j] = static_cast<unsigned long long>(m);
    in.kind[req.n_risk + j] = 1;
    need_m = true;
  }
  static_assert(sizeof(aeb_stats) % 4 == 0, "stats size");
  const long long zero_words = static_cast<long long>(L.off_zero_end / 4);
  hipLaunchKernelGGL(k_zero_u32, dim3(static_cast<unsigned>((zero_words + 255) / 256)), dim3(256),
                     0, st, reinterpret_cast<unsigned*>(base), zero_words);
  const double gstep = ng >= 2 ? (req.grid_hi - req.grid_lo) / static_cast<double>(ng - 1) : 0.0;
  hipLaunchKernelGGL(k_pass1, dim3(L.nb), dim3(EB), 0, st, out, static_cast<long long>(n), L.chunk,
                     part);
  hipLaunchKernelGGL(k_fin1, dim3(1), dim3(FB), 0, st, part, L.nb, static_cast<long long>(n),
                     out.weight ? 1 : 0, dstats, sel);
  // block histograms: the value bins only when some target needs them
  const int hw = ng >= 2 ? HG + ng + 1 : (T > 0 ? HG : 0);
  hipLaunchKernelGGL(k_pass2, dim3(L.nb2), dim3(EB), 0, st, out, static_cast<long long>(n),
                     L.chunk2, dstats, sel, need_d ? 1 : 0, need_m ? 1 : 0, req.grid_lo, gstep,
                     ng >= 2 ? 1.0 / gstep : 0.0,
                     ng, hw, bhist, vpart);
  if (hw > 0)
    hipLaunchKernelGGL(k_bin_totals, dim3((hw + 255) / 256, (L.nb2 + BT_ROWS - 1) / BT_ROWS),
                       dim3(256), 0, st, bhist, L.nb2, hw, btot);
  hipLaunchKernelGGL(k_fin2, dim3(1 + T), dim3(FB), 0, st, vpart, L.nb2,
                     static_cast<long long>(n), ng, dstats, sel, in, btot, bhist, hw, boff);
  if (out.weight) {
    hipLaunchKernelGGL(k_wpass, dim3(L.nb2), dim3(EB), 0, st, out, static_cast<long long>(n),
                       L.chunk2, req.grid_lo, gstep, ng >= 2 ? 1.0 / gstep : 0.0, ng, sel, wacc);
    hipLaunchKernelGGL(k_wfin, dim3(1), dim3(64), 0, st, static_cast<long long>(n), ng, sel, wacc,
                       dstats);
  }
  if (T > 0) {
    // the histogram pass's blocks: the offsets above are per block of it
    hipLaunchKernelGGL(k_collect, dim3(L.nb2), dim3(EB), 0, st, out, static_cast<long long>(n),
                       L.chunk2, sel, in, boff, cand);
    hipLaunchKernelGGL(k_pick, dim3(T), dim3(RB), 0, st, sel, in, cand, dstats);
  }
  AEB_HIP(hipGetLastError());
  AEB_HIP(hipMemcpyAsync(host_out, dstats, sizeof(aeb_stats), hipMemcpyDeviceToHost, st));
  return AEB_OK;
}

int reduce_fallback(const OutCols& out, int64_t n, const aeb_reduce_req& req, void* scratch_base,
                    aeb_stats* host_out, hipStream_t st) {
  // a target's value bin held more than CAP distinct candidates: radix select
  const RLayout L = layout(n, req);
  const int T = L.T;
  char* base = static_cast<char*>(scratch_base);
  aeb_stats* dstats = reinterpret_cast<aeb_stats*>(base);
  SelState* ss = reinterpret_cast<SelState*>(base + L.off_ss);
  unsigned* shist = reinterpret_cast<unsigned*>(base + L.off_sh);
  SelState rs;
  std::memset(&rs, 0, sizeof(rs));
  rs.count = T;
  for (int j = 0; j < req.n_risk; ++j) {
    long long m = static_cast<long long>(std::floor(req.risk[j] * static_cast<double>(n)));
    rs.rank[j] = static_cast<unsigned long long>(n - m - 1);
    rs.kind[j] = 0;
  }
  for (int j = 0; j < req.n_margin_q; ++j) {
    long long m = static_cast<long long>(std::floor(req.margin_q[j] * static_cast<double>(n)));
    rs.rank[req.n_risk + j] = static_cast<unsigned long long>(m);
    rs.kind[req.n_risk + j] = 1;
  }
  AEB_HIP(hipMemcpyAsync(ss, &rs, sizeof(rs), hipMemcpyHostToDevice, st));
  hipLaunchKernelGGL(k_zero_u32, dim3((T * 256 + 255) / 256), dim3(256), 0, st, shist,
                     static_cast<long long>(T * 256));
  // larger slices than the main passes: each block merges T x 256 counters
  const long long fchunk = 16384;
  const unsigned fnb = static_cast<unsigned>((n + fchunk - 1) / fchunk);
  for (int pass = 0; pass < 8; ++pass) {
    hipLaunchKernelGGL(k_select_hist, dim3(fnb), dim3(RB), 0, st, out, static_cast<long long>(n),
                       fchunk, ss, pass, shist);
    hipLaunchKernelGGL(k_select_step, dim3(1), dim3(64), 0, st, ss, pass, shist);
  }
  hipLaunchKernelGGL(k_select_out, dim3(1), dim3(64), 0, st, ss, req.n_risk, dstats);
  AEB_HIP(hipGetLastError());
  AEB_HIP(hipMemcpyAsync(host_out, dstats, sizeof(aeb_stats), hipMemcpyDeviceToHost, st));
  AEB_HIP(hipStreamSynchronize(st));
  host_out->reserved = 0;
  return AEB_OK;
}

int launch_reduce(const OutCols& out, int64_t n, const aeb_reduce_req& req, aeb_stats* host_out,
                  hipStream_t st) {
  void* base = pool_block(reduce_scratch_bytes(n, req), st);
  if (!base) return AEB_ENOMEM;
  int rc = reduce_enqueue(out, n, req, base, host_out, st);
  if (rc != AEB_OK) return rc;
  AEB_HIP(hipStreamSynchronize(st));
  const int fallback = host_out->reserved;
  host_out->reserved = 0;
  if (!fallback) return AEB_OK;
  return reduce_fallback(out, n, req, base, host_out, st);
}

}  // namespace aeb
