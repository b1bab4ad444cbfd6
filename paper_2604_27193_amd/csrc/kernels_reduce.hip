// kernels_reduce.hip -- statistics of one batch of rollout outputs (Sec. VI):
// counts and P(collision | H0) (eq. (20)), moments of the stopping distance
// (Table I), the collision-risk curve and exact minimum safe headways
// (Sec. VI-C), and margin statistics.
//
// Sums run in a fixed order (each block a fixed slice, a fixed tree inside the
// block, blocks summed in index order), so repeated calls give identical
// bits.  Order statistics are exact: a most-significant-digit radix select
// over an order-preserving map of the FP64 bit patterns, 8 passes of 8 bits,
// with per-block LDS histograms merged by integer atomics.
#include <hip/hip_runtime.h>

#include <cmath>
#include <cstring>

#include "aeb_runtime.h"

namespace aeb {

namespace {

constexpr int RB = 256;          // threads per reduction block
constexpr int MAX_T = AEB_MAX_RISK + AEB_MAX_MARGIN_Q;

struct Partial {
  long long ncol, nstop, nimp, nhor;
  double sum, dmin, dmax, msum, mmin;
  float vmax;
  float pad;
};

struct SelState {
  unsigned long long prefix[MAX_T];
  unsigned long long rank[MAX_T];
  int kind[MAX_T];   // 0: censored distance, 1: margin
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

// number of grid headways strictly below d: H0_j = lo + j * step, j < ng
__device__ inline int grid_rank(double d, double lo, double step, int ng) {
  int a = 0, b = ng;  // answer in [a, b]
  while (a < b) {
    int mid = (a + b) >> 1;
    double h = lo + static_cast<double>(mid) * step;
    if (h < d)
      a = mid + 1;
    else
      b = mid;
  }
  return a;
}

template <typename T, typename Op>
__device__ inline T block_reduce(T v, T* sh, Op op) {
  sh[threadIdx.x] = v;
  __syncthreads();
  for (int w = RB / 2; w > 0; w >>= 1) {
    if (static_cast<int>(threadIdx.x) < w) sh[threadIdx.x] = op(sh[threadIdx.x], sh[threadIdx.x + w]);
    __syncthreads();
  }
  T r = sh[0];
  __syncthreads();
  return r;
}

struct AddOp {
  template <typename T>
  __device__ T operator()(T a, T b) const { return a + b; }
};
struct MinOp {
  __device__ double operator()(double a, double b) const { return b < a ? b : a; }
};
struct MaxOp {
  __device__ double operator()(double a, double b) const { return b > a ? b : a; }
};

__global__ __launch_bounds__(RB) void k_pass1(OutCols o, long long n, long long chunk, double glo,
                                              double gstep, int ng, unsigned* ghist, Partial* part) {
  __shared__ double shd[RB];
  __shared__ long long shl[RB];
  __shared__ unsigned hist[AEB_MAX_GRID + 1];
  for (int j = threadIdx.x; j <= ng; j += RB) hist[j] = 0;
  __syncthreads();
  const long long lo = static_cast<long long>(blockIdx.x) * chunk;
  const long long hi = lo + chunk < n ? lo + chunk : n;
  long long ncol = 0, nstop = 0, nimp = 0, nhor = 0;
  double sum = 0.0, dmin = INFINITY, dmax = -INFINITY, msum = 0.0, mmin = INFINITY;
  float vmax = 0.0f;
  for (long long i = lo + threadIdx.x; i < hi; i += RB) {
    const uint8_t st = o.status[i];
    const double d = o.dist[i];
    const double m = o.margin[i];
    const int end = st & 3;
    if (st & AEB_COLLIDED) {
      ++ncol;
      const float vi = o.vimp[i];
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
    if (ng >= 2) {
      const double dc = end == AEB_END_STOP ? d : INFINITY;
      atomicAdd(&hist[grid_rank(dc, glo, gstep, ng)], 1u);
    }
  }
  Partial p;
  p.ncol = block_reduce(ncol, shl, AddOp());
  p.nstop = block_reduce(nstop, shl, AddOp());
  p.nimp = block_reduce(nimp, shl, AddOp());
  p.nhor = block_reduce(nhor, shl, AddOp());
  p.sum = block_reduce(sum, shd, AddOp());
  p.dmin = block_reduce(dmin, shd, MinOp());
  p.dmax = block_reduce(dmax, shd, MaxOp());
  p.msum = block_reduce(msum, shd, AddOp());
  p.mmin = block_reduce(mmin, shd, MinOp());
  p.vmax = static_cast<float>(block_reduce(static_cast<double>(vmax), shd, MaxOp()));
  p.pad = 0.0f;
  if (threadIdx.x == 0) part[blockIdx.x] = p;
  if (ng >= 2) {
    for (int j = threadIdx.x; j <= ng; j += RB)
      if (hist[j]) atomicAdd(&ghist[j], hist[j]);
  }
}

__global__ void k_finalize1(const Partial* part, int nb, long long n, int ng,
                            const unsigned* ghist, aeb_stats* st) {
  if (threadIdx.x != 0 || blockIdx.x != 0) return;
  long long ncol = 0, nstop = 0, nimp = 0, nhor = 0;
  double sum = 0.0, dmin = INFINITY, dmax = -INFINITY, msum = 0.0, mmin = INFINITY;
  float vmax = 0.0f;
  for (int b = 0; b < nb; ++b) {
    const Partial& p = part[b];
    ncol += p.ncol;
    nstop += p.nstop;
    nimp += p.nimp;
    nhor += p.nhor;
    sum += p.sum;
    dmin = p.dmin < dmin ? p.dmin : dmin;
    dmax = p.dmax > dmax ? p.dmax : dmax;
    msum += p.msum;
    mmin = p.mmin < mmin ? p.mmin : mmin;
    vmax = p.vmax > vmax ? p.vmax : vmax;
  }
  st->n = n;
  st->n_collide = ncol;
  st->n_stop = nstop;
  st->n_impact = nimp;
  st->n_horizon = nhor;
  st->p_collision = static_cast<double>(ncol) / static_cast<double>(n);
  st->mean_dist = nstop > 0 ? sum / static_cast<double>(nstop) : NAN;
  st->dist_min = nstop > 0 ? dmin : NAN;
  st->dist_max = nstop > 0 ? dmax : NAN;
  st->sd_dist = NAN;
  st->margin_min = mmin;
  st->margin_mean = msum / static_cast<double>(n);
  st->v_impact_max = vmax;
  // risk curve: #{D > H0_j} = #{D whose grid rank exceeds j}
  long long above = n;
  for (int j = 0; j < ng; ++j) {
    above -= ghist[j];
    st->risk_count[j] = above;
    st->risk_p[j] = static_cast<double>(above) / static_cast<double>(n);
  }
}

__global__ __launch_bounds__(RB) void k_pass2(OutCols o, long long n, long long chunk,
                                              const aeb_stats* st, double* part) {
  __shared__ double shd[RB];
  const double mean = st->mean_dist;
  const long long lo = static_cast<long long>(blockIdx.x) * chunk;
  const long long hi = lo + chunk < n ? lo + chunk : n;
  double ss = 0.0;
  for (long long i = lo + threadIdx.x; i < hi; i += RB) {
    if ((o.status[i] & 3) == AEB_END_STOP) {
      const double e = o.dist[i] - mean;
      ss += e * e;
    }
  }
  ss = block_reduce(ss, shd, AddOp());
  if (threadIdx.x == 0) part[blockIdx.x] = ss;
}

__global__ void k_finalize2(const double* part, int nb, aeb_stats* st) {
  if (threadIdx.x != 0 || blockIdx.x != 0) return;
  double ss = 0.0;
  for (int b = 0; b < nb; ++b) ss += part[b];
  st->sd_dist = st->n_stop > 1 ? sqrt(ss / static_cast<double>(st->n_stop - 1)) : NAN;
}

// one radix digit for every select target
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
  bool need_d = false, need_m = false;
  for (int t = 0; t < T; ++t) (kind[t] ? need_m : need_d) = true;
  const long long lo = static_cast<long long>(blockIdx.x) * chunk;
  const long long hi = lo + chunk < n ? lo + chunk : n;
  for (long long i = lo + threadIdx.x; i < hi; i += RB) {
    const unsigned long long kd = need_d ? ordered(censored(o.dist, o.status, i)) : 0ull;
    const unsigned long long km = need_m ? ordered(o.margin[i]) : 0ull;
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

__global__ void k_zero_u32(unsigned* p, long long n) {
  long long i = static_cast<long long>(blockIdx.x) * blockDim.x + threadIdx.x;
  if (i < n) p[i] = 0u;
}

size_t align256(size_t b) { return (b + 255) & ~size_t(255); }

}  // namespace

int launch_reduce(const OutCols& out, int64_t n, const aeb_reduce_req& req, aeb_stats* host_out,
                  hipStream_t st) {
  const long long chunk = n <= 65536 ? 1024 : 4096;
  const int nb = static_cast<int>((n + chunk - 1) / chunk);
  const int ng = req.n_grid;
  const int T = req.n_risk + req.n_margin_q;
  // scratch layout
  size_t off_part = 0;
  size_t off_var = align256(off_part + sizeof(Partial) * nb);
  size_t off_stats = align256(off_var + sizeof(double) * nb);
  size_t off_rh = align256(off_stats + sizeof(aeb_stats));
  size_t off_ss = align256(off_rh + sizeof(unsigned) * (AEB_MAX_GRID + 1));
  size_t off_sh = align256(off_ss + sizeof(SelState));
  size_t total = align256(off_sh + sizeof(unsigned) * MAX_T * 256);
  char* base = static_cast<char*>(scratch(total, st));
  if (!base) return AEB_ENOMEM;
  Partial* part = reinterpret_cast<Partial*>(base + off_part);
  double* vpart = reinterpret_cast<double*>(base + off_var);
  aeb_stats* dstats = reinterpret_cast<aeb_stats*>(base + off_stats);
  unsigned* rhist = reinterpret_cast<unsigned*>(base + off_rh);
  SelState* ss = reinterpret_cast<SelState*>(base + off_ss);
  unsigned* shist = reinterpret_cast<unsigned*>(base + off_sh);

  // select targets: ranks computed exactly as floor(level * N) in binary64
  SelState hs;
  std::memset(&hs, 0, sizeof(hs));
  hs.count = T;
  for (int j = 0; j < req.n_risk; ++j) {
    long long m = static_cast<long long>(std::floor(req.risk[j] * static_cast<double>(n)));
    hs.rank[j] = static_cast<unsigned long long>(n - m - 1);
    hs.kind[j] = 0;
  }
  for (int j = 0; j < req.n_margin_q; ++j) {
    long long m = static_cast<long long>(std::floor(req.margin_q[j] * static_cast<double>(n)));
    hs.rank[req.n_risk + j] = static_cast<unsigned long long>(m);
    hs.kind[req.n_risk + j] = 1;
  }
  AEB_HIP(hipMemcpyAsync(ss, &hs, sizeof(hs), hipMemcpyHostToDevice, st));
  hipLaunchKernelGGL(k_zero_u32, dim3((AEB_MAX_GRID + 1 + 255) / 256), dim3(256), 0, st, rhist,
                     static_cast<long long>(AEB_MAX_GRID + 1));
  hipLaunchKernelGGL(k_zero_u32, dim3((MAX_T * 256 + 255) / 256), dim3(256), 0, st, shist,
                     static_cast<long long>(MAX_T * 256));
  AEB_HIP(hipMemsetAsync(dstats, 0, sizeof(aeb_stats), st));
  const double gstep = ng >= 2 ? (req.grid_hi - req.grid_lo) / static_cast<double>(ng - 1) : 0.0;
  hipLaunchKernelGGL(k_pass1, dim3(nb), dim3(RB), 0, st, out, static_cast<long long>(n), chunk,
                     req.grid_lo, gstep, ng, rhist, part);
  hipLaunchKernelGGL(k_finalize1, dim3(1), dim3(64), 0, st, part, nb, static_cast<long long>(n), ng,
                     rhist, dstats);
  hipLaunchKernelGGL(k_pass2, dim3(nb), dim3(RB), 0, st, out, static_cast<long long>(n), chunk,
                     dstats, vpart);
  hipLaunchKernelGGL(k_finalize2, dim3(1), dim3(64), 0, st, vpart, nb, dstats);
  if (T > 0) {
    for (int pass = 0; pass < 8; ++pass) {
      hipLaunchKernelGGL(k_select_hist, dim3(nb), dim3(RB), 0, st, out, static_cast<long long>(n),
                         chunk, ss, pass, shist);
      hipLaunchKernelGGL(k_select_step, dim3(1), dim3(64), 0, st, ss, pass, shist);
    }
    hipLaunchKernelGGL(k_select_out, dim3(1), dim3(64), 0, st, ss, req.n_risk, dstats);
  }
  AEB_HIP(hipGetLastError());
  AEB_HIP(hipMemcpyAsync(host_out, dstats, sizeof(aeb_stats), hipMemcpyDeviceToHost, st));
  AEB_HIP(hipStreamSynchronize(st));
  return AEB_OK;
}

}  // namespace aeb
