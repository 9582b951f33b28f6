// Singular value decomposition of the quantum-number blocks on gfx950.
//
// One-sided Jacobi: the shorter side of an R x C block (columns if R >= C,
// else rows) is rotated pairwise until the vectors are mutually orthogonal to
// rounding; their norms are the singular values.  No rotation matrix is
// accumulated.  The kernels write the rotated vectors sorted by decreasing
// norm (columns case: U = x / s, rows case: B = x = s v^T) and the singular
// values; k_svd_factor then forms the other factor of the kept vectors from
// one product with the block (B = U^T T, or U = T B^T / s^2).
//
// Pair ordering (k_jacobi).  n vectors are held by P = ceil(n/2) processors
// (aligned groups of G lanes of one wave).  Each processor keeps one resident
// vector in registers; the other floor(n/2) vectors are travellers in LDS
// slots.  A node of the ordering has r residents and t travellers
// (|r - t| <= 1) and pairs every resident with every traveller in max(r, t)
// rounds (resident k meets traveller (k + round) mod max(r, t)).  It then
// splits: the residents form one child, the travellers the other, and x of
// the processors swap their resident with one traveller slot each, so that
// every child again has residents in registers and travellers in LDS.  After
// ceil(log2 n) levels every pair has met exactly once (one sweep) with about
// n rounds; per rotation only the traveller moves through LDS.  Lane gl of a
// processor holds the E components gl*E .. gl*E+E-1 of a vector (zero past
// the end), so every inner loop has a compile-time trip count.
#include <hip/hip_runtime.h>

#include "internal.hpp"

namespace tnqe {

namespace {

// one 64-bit value moved by a DPP lane permutation (two 32-bit moves)
template <int CTRL>
__device__ inline double dpp64(double v) {
  const long long x = __double_as_longlong(v);
  const int lo = __builtin_amdgcn_update_dpp(0, (int)(x & 0xffffffffll), CTRL, 0xF, 0xF, false);
  const int hi = __builtin_amdgcn_update_dpp(0, (int)(x >> 32), CTRL, 0xF, 0xF, false);
  return __longlong_as_double(((long long)hi << 32) | (unsigned int)lo);
}

// Sum over an aligned group of G lanes (G a power of two <= 64).  Every lane
// of the group ends with the same bits: each step adds two lanes' partial
// sums, and the two lanes of a step add the same operands.
__device__ inline double group_sum(double v, int G) {
  if (G >= 2) v += dpp64<0xB1>(v);    // quad_perm [1,0,3,2]: lane ^ 1
  if (G >= 4) v += dpp64<0x4E>(v);    // quad_perm [2,3,0,1]: lane ^ 2
  if (G >= 8) v += dpp64<0x141>(v);   // row_half_mirror: the other quad of 8
  if (G >= 16) v += dpp64<0x140>(v);  // row_mirror: the other half of 16
  if (G >= 32) v += __shfl_xor(v, 16, 64);
  if (G >= 64) v += __shfl_xor(v, 32, 64);
  return v;
}

__device__ inline double wave_sum(double v) {
  for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o, 64);
  return v;
}

// 1/sqrt(x) and 1/x for normal positive x: the hardware estimates (24 bits,
// measured on gfx950) refined by NS Newton steps (each doubles the bits: one
// step gives ~2e-15, two reach rounding level).
template <int NS>
__device__ inline double rsqrt_nr(double x) {
  double y = __builtin_amdgcn_rsq(x);
  const double hx = 0.5 * x;
#pragma unroll
  for (int i = 0; i < NS; ++i) y = y * fma(-hx * y, y, 1.5);
  return y;
}
template <int NS>
__device__ inline double rcp_nr(double x) {
  double y = __builtin_amdgcn_rcp(x);
#pragma unroll
  for (int i = 0; i < NS; ++i) y = fma(y, fma(-x, y, 1.0), y);
  return y;
}

// Rotation that orthogonalises (x, y) with squared norms al, be and product
// ga != 0: x' = c x - s y, y' = s x + c y; returns tan (for the norm updates).
// tan is the smaller root of t^2 ga + t (be - al) - ga = 0, written without
// cancellation; c = 1/sqrt(1 + t^2), s = c t.  Only c needs rounding-level
// accuracy (c^2 + s^2 = 1 keeps the norms); an error of ~1e-15 in t merely
// leaves a residual inner product of that relative size, far below the
// convergence threshold, so t takes one Newton step per estimate.
__device__ inline double jacobi_angle(double al, double be, double ga, double &c, double &s) {
  const double d = be - al;
  const double q = fma(d, d, 4.0 * ga * ga);
  const double r = q * rsqrt_nr<1>(q);   // sqrt(d^2 + 4 ga^2)
  const double t = (d >= 0.0 ? 2.0 * ga : -2.0 * ga) * rcp_nr<1>(fabs(d) + r);
  c = rsqrt_nr<2>(fma(t, t, 1.0));
  s = c * t;
  return t;
}

// sum of squares / dot product of E register elements, four partial sums
// E doubles of a 16-byte aligned LDS chunk, as 128-bit accesses
template <int E>
__device__ inline void ld_chunk(const double *p, double (&x)[E]) {
#pragma unroll
  for (int e = 0; e < E; e += 2) {
    const double2 v = reinterpret_cast<const double2 *>(p)[e >> 1];
    x[e] = v.x;
    x[e + 1] = v.y;
  }
}
template <int E>
__device__ inline void st_chunk(double *p, const double (&x)[E]) {
#pragma unroll
  for (int e = 0; e < E; e += 2) reinterpret_cast<double2 *>(p)[e >> 1] = make_double2(x[e], x[e + 1]);
}

template <int E>
__device__ inline double dot_e(const double (&x)[E], const double (&y)[E]) {
  double p[4] = {0.0, 0.0, 0.0, 0.0};
#pragma unroll
  for (int e = 0; e < E; ++e) p[e & 3] = fma(x[e], y[e], p[e & 3]);
  return (p[0] + p[1]) + (p[2] + p[3]);
}

// rank of value i among n (descending, ties by index)
__device__ inline int rank_of(const double *sig, int n, int i) {
  const double si = sig[i];
  int r = 0;
  for (int j = 0; j < n; ++j) {
    const double sj = sig[j];
    r += (sj > si || (sj == si && j < i)) ? 1 : 0;
  }
  return r;
}

// squared relative inner product above which a rotation keeps the sweeps going
constexpr double kBig2 = 1e-20;

// at most 1024 threads (E <= 20) or 768 (E = 24, for the register budget).
// Waves per SIMD the register allocation must allow: 6 for E = 8 and 5 for
// E = 12 (80 and 96 registers; the few values that then leave the registers
// are reloaded once per sweep, outside the rotation rounds), so that two
// workgroups of 768 threads, or three of 512, share a compute unit.
template <int E>
constexpr int jacobi_waves_per_simd() {
  return E == 8 ? 6 : E == 12 ? 5 : 1;
}
template <int E>
__global__ void __launch_bounds__(E > 20 ? 768 : 1024) __attribute__((amdgpu_waves_per_eu(jacobi_waves_per_simd<E>())))
k_jacobi(const Blk *blks, const int *idx, double *scratch, int max_sweeps, int *sweeps_out) {
  extern __shared__ __align__(16) double lds[];
  const Blk b = blks[idx[blockIdx.x]];
  const int R = b.R, C = b.C;
  const bool cols = R >= C;
  const int n = b.n, m = cols ? R : C;
  if (n == 0) return;
  // in an LDS row the chunk of lane gl starts at gl*SL doubles; SL = E + 2
  // keeps every chunk 16-byte aligned (128-bit LDS accesses) and spreads the
  // chunks of 8 consecutive lanes over all 32 four-byte banks
  constexpr int SL = E + 2;
  static_assert(E % 4 == 0, "E");
  const int G = b.grp, mp = G * SL;
  const int P = (n + 1) >> 1, NTr = n >> 1;
  double *X = lds;                              // traveller rows [NTr][mp]
  double *tnrm = X + (int64_t)NTr * mp;         // traveller squared norms
  double *sig = tnrm + NTr;                     // singular values [n]
  int *rnk = reinterpret_cast<int *>(sig + n);  // ranks [n]
  __shared__ int s_rot[2], s_big[2];
  __shared__ unsigned long long s_amax;
  const double *T = scratch + b.offT;
  const int p = threadIdx.x / G, gl = threadIdx.x - p * G;
  const bool act = p < P;
  const int l0 = gl * E;
  double *Xl = X + gl * SL;                     // this lane's chunk of row 0
  double res[E], trv[E];
  // vector i of the block: component l at T[i * vs + l * ls]
  const int64_t vs = cols ? 1 : C, ls = cols ? C : 1;
  if (act) {
    const double *src = T + (int64_t)p * vs + (int64_t)l0 * ls;
#pragma unroll
    for (int e = 0; e < E; ++e) {
      res[e] = l0 + e < m ? src[e * ls] : 0.0;
      __builtin_amdgcn_sched_barrier(0);
    }
    if (p < NTr) {
      const double *tsrc = T + (int64_t)(P + p) * vs + (int64_t)l0 * ls;
      for (int e = 0; e < E; ++e) Xl[p * mp + e] = l0 + e < m ? tsrc[e * ls] : 0.0;
    }
  }
  if (threadIdx.x == 0) {
    s_rot[0] = s_rot[1] = 0;
    s_big[0] = s_big[1] = 0;
  }
  __syncthreads();
  // rounding floor of a length-m dot product relative to the norms (squared)
  const double tol = fmax(1e-15, 2.3e-16 * sqrt((double)m)), tol2 = tol * tol;
  double rn = 0.0;   // squared norm of the resident (same in all lanes of the group)
  int sweep = 0;
  for (; sweep < max_sweeps && n > 1; ++sweep) {
    const int fl = sweep & 1;
    if (threadIdx.x == 0) s_amax = 0ull;
    __syncthreads();
    // squared norms, recomputed each sweep and updated exactly per rotation
    if (act) {
      rn = group_sum(dot_e(res, res), G);
      double mx = rn;
      if (p < NTr) {
        ld_chunk<E>(Xl + p * mp, trv);
        const double t2 = group_sum(dot_e(trv, trv), G);
        if (gl == 0) tnrm[p] = t2;
        mx = fmax(mx, t2);
      }
      if (gl == 0) atomicMax(&s_amax, (unsigned long long)__double_as_longlong(mx));   // >= 0 orders as an integer
    }
    // vectors placed by decreasing norm: the larger half resident (processor
    // p holds the p-th largest), the smaller half in the traveller slots, so
    // that each sweep first rotates every large vector against every small
    // one (about a fifth fewer sweeps on the gate blocks).  The vectors pass,
    // in sorted order, through rows of G E doubles (each lane's chunk whole,
    // no bounds checks) laid over the U and B areas, unused until the end;
    // blocks whose areas cannot hold the padded rows keep their placement.
    const bool sorted = b.offB >= b.offU && (int64_t)n * G * E <= (b.offB - b.offU) + (int64_t)n * C;
    if (sorted) {
      if (act && gl == 0) sig[p] = rn;
      __syncthreads();   // every traveller norm written
      for (int i = threadIdx.x; i < NTr; i += blockDim.x) sig[P + i] = tnrm[i];
      __syncthreads();
      for (int i = threadIdx.x; i < n; i += blockDim.x) rnk[i] = rank_of(sig, n, i);
      __syncthreads();
      double *stage = scratch + b.offU + l0, *snrm = scratch + b.offS;
      const int64_t rs = (int64_t)G * E;
      if (act) {
        const int rr = rnk[p];
        st_chunk<E>(stage + rr * rs, res);
        if (gl == 0) snrm[rr] = rn;
        if (p < NTr) {
          const int rt = rnk[P + p];
          st_chunk<E>(stage + rt * rs, trv);
          if (gl == 0) snrm[rt] = tnrm[p];
        }
      }
      __syncthreads();
      if (act) {
        ld_chunk<E>(stage + p * rs, res);
        rn = snrm[p];
        if (p < NTr) {
          ld_chunk<E>(stage + (P + p) * rs, trv);
          st_chunk<E>(Xl + p * mp, trv);
          if (gl == 0) tnrm[p] = snrm[P + p];
        }
      }
    }
    __syncthreads();
    // vectors below 1e-14 of the largest are rounding noise of a rank-deficient
    // block: they are not rotated (they never survive a truncation)
    const double tiny = __longlong_as_double((long long)s_amax) * 1e-28;
    int rotated = 0, big = 0;
    int pb = 0, sb = 0, r = P, t = NTr;   // this processor's node
    for (int lv = 0;; ++lv) {
      if (((n + (1 << lv) - 1) >> lv) <= 1) break;            // largest node has one vector
      const int rounds = (n + (2 << lv) - 1) >> (lv + 1);      // = max over nodes of max(r, t)
      const int k = p - pb, q = max(r, t);
      for (int rho = 0; rho < rounds; ++rho) {
        if (act && rho < q) {
          int j = k + rho;
          if (j >= q) j -= q;
          if (j < t) {
            double *xs = Xl + (sb + j) * mp;
            ld_chunk<E>(xs, trv);
            const double al = rn, be = tnrm[sb + j];
            if (al > tiny && be > tiny) {
              const double ga = group_sum(dot_e(res, trv), G);
              if (ga * ga > tol2 * (al * be)) {
                big |= ga * ga > kBig2 * (al * be) ? 1 : 0;
                double c, s;
                const double tn = jacobi_angle(al, be, ga, c, s);
                // one component at a time (keeps the live registers at the
                // two vectors; the stores retire the traveller as it goes)
#pragma unroll
                for (int e = 0; e < E; e += 2) {
                  const double u0 = res[e], v0 = trv[e], u1 = res[e + 1], v1 = trv[e + 1];
                  res[e] = c * u0 - s * v0;
                  res[e + 1] = c * u1 - s * v1;
                  reinterpret_cast<double2 *>(xs)[e >> 1] = make_double2(s * u0 + c * v0, s * u1 + c * v1);
                  __builtin_amdgcn_sched_barrier(0);
                }
                rn = fmax(al - tn * ga, 0.0);
                if (gl == 0) tnrm[sb + j] = be + tn * ga;
                rotated = 1;
              }
            }
          }
        }
        __syncthreads();
      }
      // split the node: residents (pb .. pb+rA) stay, the next x processors
      // swap their resident with the traveller in slot sb + (k - rA)
      const int x = (t == r + 1) ? (r + 1) >> 1 : r >> 1;
      const int rA = r - x;
      const bool sw = act && k >= rA && k < r;
      double *xw = Xl + (sb + (k - rA)) * mp;
      double nn = 0.0;
      if (sw) {
        ld_chunk<E>(xw, trv);
        nn = tnrm[sb + (k - rA)];
      }
      __syncthreads();
      if (sw) {
        st_chunk<E>(xw, res);
#pragma unroll
        for (int e = 0; e < E; ++e) res[e] = trv[e];
        if (gl == 0) tnrm[sb + (k - rA)] = rn;
        rn = nn;
      }
      __syncthreads();
      if (k < rA) {
        r = rA;
        t = x;
      } else {
        pb += rA;
        sb += x;
        t = t - x;
        r = x;
      }
    }
    if (rotated && gl == 0) atomicOr(&s_rot[fl], 1);
    if (big && gl == 0) atomicOr(&s_big[fl], 1);
    __syncthreads();
    const int any = s_rot[fl], any_big = s_big[fl];
    // the other flags are cleared only after every thread has read these
    if (threadIdx.x == 0) s_rot[fl ^ 1] = s_big[fl ^ 1] = 0;
    // converged: no rotation, or only rotations of pairs already orthogonal
    // to 1e-10 (what they leave is of second order, ~1e-20, far below tol)
    if (any == 0 || any_big == 0) break;
  }
  if (sweeps_out && threadIdx.x == 0) sweeps_out[idx[blockIdx.x]] = sweep;
  // singular values from the final vectors (residents 0..P, travellers P..n)
  if (act) {
    double s2 = 0.0;
#pragma unroll
    for (int e = 0; e < E; ++e) s2 += res[e] * res[e];
    s2 = group_sum(s2, G);
    if (gl == 0) sig[p] = sqrt(s2);
    if (p < NTr) {
      double t2 = 0.0;
#pragma unroll
      for (int e = 0; e < E; ++e) {
        const double v = Xl[p * mp + e];
        t2 += v * v;
      }
      t2 = group_sum(t2, G);
      if (gl == 0) sig[P + p] = sqrt(t2);
    }
  }
  __syncthreads();
  double *S = scratch + b.offS;
  for (int i = threadIdx.x; i < n; i += blockDim.x) {
    const int rk = rank_of(sig, n, i);
    rnk[i] = rk;
    S[rk] = sig[i];
  }
  __syncthreads();
  // sorted vectors: U[rank] = x / s (columns), B[rank] = x (rows); U is stored
  // by column ([n][R]), B by row ([n][C]), so both are rows of length m here
  double *out = scratch + (cols ? b.offU : b.offB);
  if (act) {
    const int rk = rnk[p];
    const double sp = sig[p];
#pragma unroll
    for (int e = 0; e < E; ++e) {
      const int l = l0 + e;
      if (l < m) out[(int64_t)rk * m + l] = cols ? (sp > 0.0 ? res[e] / sp : 0.0) : res[e];
    }
    if (p < NTr) {
      const int rt = rnk[P + p];
      const double st = sig[P + p];
#pragma unroll
      for (int e = 0; e < E; ++e) {
        const int l = l0 + e;
        if (l < m) {
          const double v = Xl[p * mp + e];
          out[(int64_t)rt * m + l] = cols ? (st > 0.0 ? v / st : 0.0) : v;
        }
      }
    }
  }
}

// Blocks too large for k_jacobi: the vectors live in a global work area and
// are rotated in cyclic round-robin order by groups of G lanes (same output).
// mode kJwFull runs everything in this workgroup; kJwLoad only fills the work
// area (and clears the control words ctl of the chip-wide variant), kJwFinish
// only takes the final norms, ranks and writes the vectors after `sweeps_done`
// sweeps made by k_jw_norms with k_jw_round or k_jwb_round.
__global__ void __launch_bounds__(1024) k_jacobi_global(const Blk *blks, const int *idx, double *scratch,
                                                        int max_sweeps, int *sweeps_out, int mode,
                                                        int sweeps_done, unsigned long long *ctl) {
  constexpr int NT = 1024, NW = NT / 64;
  const Blk b = blks[idx[blockIdx.x]];
  const int R = b.R, C = b.C;
  const bool cols = R >= C;
  const int n = b.n, m = cols ? R : C;
  if (n == 0) return;
  double *X = scratch + b.offW;                 // X[i*m + l]: vector i
  double *sig = X + (int64_t)n * m;
  __shared__ int s_rot[2], s_big[2];
  __shared__ unsigned long long s_amax;
  const double *T = scratch + b.offT;
  if (threadIdx.x == 0) {
    s_rot[0] = s_rot[1] = 0;
    s_big[0] = s_big[1] = 0;
  }
  if (mode != kJwFinish) {
    for (int64_t e = threadIdx.x; e < (int64_t)n * m; e += NT) {
      const int i = e / m, l = e - (int64_t)i * m;
      X[e] = cols ? T[(int64_t)l * C + i] : T[(int64_t)i * C + l];
    }
    if (mode == kJwLoad) {
      if (threadIdx.x < 4) ctl[threadIdx.x] = 0ull;
      return;
    }
  }
  __syncthreads();
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const int G = 64, ngroup = NT / G, grp = threadIdx.x / G, gl = threadIdx.x % G;
  const int np = n + (n & 1);
  const double tol = fmax(1e-15, 2.3e-16 * sqrt((double)m));
  int sweep = mode == kJwFinish ? sweeps_done : 0;
  for (; mode == kJwFull && sweep < max_sweeps && n > 1; ++sweep) {
    const int fl = sweep & 1;
    int rotated = 0, big = 0;
    if (threadIdx.x == 0) s_amax = 0ull;
    __syncthreads();
    for (int i = grp; i < n; i += ngroup) {
      double s2 = 0.0;
      for (int l = gl; l < m; l += G) s2 += X[(int64_t)i * m + l] * X[(int64_t)i * m + l];
      s2 = wave_sum(s2);
      if (gl == 0) {
        sig[i] = s2;
        atomicMax(&s_amax, (unsigned long long)__double_as_longlong(s2));
      }
    }
    __syncthreads();
    const double tiny = __longlong_as_double((long long)s_amax) * 1e-28;
    for (int rd = 0; rd < np - 1; ++rd) {
      for (int k = grp; k < np / 2; k += ngroup) {
        int i, j;
        if (k == 0) {
          i = np - 1;
          j = rd;
        } else {
          i = (rd + k) % (np - 1);
          j = (rd - k + np - 1) % (np - 1);
        }
        if (i >= n || j >= n) continue;
        const double al = sig[i], be = sig[j];
        if (al <= tiny || be <= tiny) continue;
        double *xi = X + (int64_t)i * m, *xj = X + (int64_t)j * m;
        double ga = 0.0;
        for (int l = gl; l < m; l += G) ga += xi[l] * xj[l];
        ga = wave_sum(ga);
        if (fabs(ga) <= tol * sqrt(al * be)) continue;
        big |= ga * ga > kBig2 * (al * be) ? 1 : 0;
        double c, s;
        const double tn = jacobi_angle(al, be, ga, c, s);
        for (int l = gl; l < m; l += G) {
          const double u = xi[l], v = xj[l];
          xi[l] = c * u - s * v;
          xj[l] = s * u + c * v;
        }
        if (gl == 0) {
          sig[i] = fmax(al - tn * ga, 0.0);
          sig[j] = be + tn * ga;
        }
        rotated = 1;
      }
      __syncthreads();
    }
    if (rotated) atomicOr(&s_rot[fl], 1);
    if (big) atomicOr(&s_big[fl], 1);
    __syncthreads();
    const int any = s_rot[fl], any_big = s_big[fl];
    if (threadIdx.x == 0) s_rot[fl ^ 1] = s_big[fl ^ 1] = 0;
    // converged as in k_jacobi: no rotation, or only rotations of pairs
    // already orthogonal to 1e-10
    if (any == 0 || any_big == 0) break;
  }
  if (sweeps_out && threadIdx.x == 0) sweeps_out[idx[blockIdx.x]] = sweep;
  for (int i = wave; i < n; i += NW) {
    double s2 = 0.0;
    for (int l = lane; l < m; l += 64) s2 += X[(int64_t)i * m + l] * X[(int64_t)i * m + l];
    s2 = wave_sum(s2);
    if (lane == 0) sig[i] = sqrt(s2);
  }
  __syncthreads();
  __shared__ int s_rank[1024];
  double *S = scratch + b.offS;
  for (int i = threadIdx.x; i < n; i += NT) {
    const int rk = rank_of(sig, n, i);
    s_rank[i] = rk;
    S[rk] = sig[i];
  }
  __syncthreads();
  double *out = scratch + (cols ? b.offU : b.offB);
  for (int64_t e = threadIdx.x; e < (int64_t)n * m; e += NT) {
    const int i = e / m, l = e - (int64_t)i * m;
    const double si = sig[i];
    out[(int64_t)s_rank[i] * m + l] = cols ? (si > 0.0 ? X[e] / si : 0.0) : X[e];
  }
}

// The factor not produced by the Jacobi kernels, for the first `kept` sorted
// vectors: columns case B[j][c] = sum_r U[j][r] T[r][c]; rows case
// U[j][r] = sum_c B[j][c] T[r][c] / s_j^2.  One 64 x 64 output tile per
// workgroup, 4 x 4 per thread, K staged through LDS in steps of 16 (the next
// step's loads issued before the current step's products).
constexpr int kFT = 64, kFK = 16;
__global__ void __launch_bounds__(256) k_svd_factor(const Blk *blks, Units un, double *scratch) {
  const int bi = find_unit(un.first, un.n, blockIdx.x);
  const Blk b = blks[bi];
  const int I = b.kept;
  const bool cols = b.R >= b.C;
  const double *T = scratch + b.offT;
  const double *S = scratch + b.offS;
  // out[i][j] = sc_i * sum_k A[i][k] * Bm(k, j)
  const double *A = scratch + (cols ? b.offU : b.offB);
  double *out = scratch + (cols ? b.offB : b.offU);
  const int K = cols ? b.R : b.C, J = cols ? b.C : b.R;
  // Bm(k, j) = T[k][j] (columns case) or T[j][k] (rows case)
  const int64_t bk = cols ? b.C : 1, bj = cols ? 1 : b.C;
  __shared__ double As[kFK][kFT + 1];
  __shared__ double Bs[kFK][kFT + 1];
  const int tx = threadIdx.x & 15, ty = threadIdx.x >> 4;
  static_assert(kFT == kGateTile, "tile");
  const int tilesJ = (J + kFT - 1) / kFT;
  {
    const int tile = blockIdx.x - un.first[bi];
    const int i0 = (tile / tilesJ) * kFT, j0 = (tile % tilesJ) * kFT;
    if (i0 >= I) return;   // units are counted for all n vectors
    double acc[4][4] = {};
    // the next K chunk's operands are loaded into registers while the
    // current chunk is multiplied
    constexpr int RF = kFK * kFT / 256;
    double ra[RF], rb[RF];
    auto fetch = [&](int k0) {
#pragma unroll
      for (int u = 0; u < RF; ++u) {
        const int e = threadIdx.x + 256 * u;
        // A tile: 64 rows i x 16 k (k fastest: A rows are contiguous in k)
        const int ii = e / kFK, kk = e % kFK;
        const int gi = i0 + ii, gk = k0 + kk;
        ra[u] = (gi < I && gk < K) ? A[(int64_t)gi * K + gk] : 0.0;
        // B tile: 16 k x 64 j, with the contiguous index fastest
        const int kb = cols ? e / kFT : e % kFK, jj = cols ? e % kFT : e / kFK;
        const int gj = j0 + jj, gk2 = k0 + kb;
        rb[u] = (gj < J && gk2 < K) ? T[(int64_t)gk2 * bk + (int64_t)gj * bj] : 0.0;
      }
    };
    if (K > 0) fetch(0);
    for (int k0 = 0; k0 < K; k0 += kFK) {
#pragma unroll
      for (int u = 0; u < RF; ++u) {
        const int e = threadIdx.x + 256 * u;
        As[e % kFK][e / kFK] = ra[u];
        if (cols) Bs[e / kFT][e % kFT] = rb[u];
        else Bs[e % kFK][e / kFK] = rb[u];
      }
      __syncthreads();
      if (k0 + kFK < K) fetch(k0 + kFK);
#pragma unroll
      for (int kk = 0; kk < kFK; ++kk) {
        double a[4], bv[4];
#pragma unroll
        for (int u = 0; u < 4; ++u) {
          a[u] = As[kk][ty + 16 * u];
          bv[u] = Bs[kk][tx + 16 * u];
        }
#pragma unroll
        for (int u = 0; u < 4; ++u)
#pragma unroll
          for (int v = 0; v < 4; ++v) acc[u][v] += a[u] * bv[v];
      }
      __syncthreads();
    }
#pragma unroll
    for (int u = 0; u < 4; ++u) {
      const int gi = i0 + ty + 16 * u;
      if (gi >= I) continue;
      double sc = 1.0;
      if (!cols) {
        const double s = S[gi];
        sc = s > 0.0 ? 1.0 / (s * s) : 0.0;
      }
#pragma unroll
      for (int v = 0; v < 4; ++v) {
        const int gj = j0 + tx + 16 * v;
        if (gj < J) out[(int64_t)gi * J + gj] = acc[u][v] * sc;
      }
    }
  }
}

// The sweeps of k_jacobi_global spread over the chip for one wide block (the
// dense eigenproblems of the generalized sweep are 400 and more columns wide,
// and one workgroup then waits on its own loads most of the time).  A sweep is
// one k_jw_norms launch and one k_jw_round launch per round of the
// round-robin ordering, one wave per pair; the kernel boundaries order the
// rounds.  Lane partition, sums, angles and norm updates are those of
// k_jacobi_global, so both give the same bits.  Control words: ctl[slot] the
// sweep's largest squared norm (as bits), ctl[2 + slot] bit 0 set when a pair
// of the sweep rotated, bit 1 when one was not yet orthogonal to 1e-10 (the
// sweeps end at the first sweep without such a rotation, as in
// k_jacobi_global); sweep s uses slot s & 1 and clears the other slot.
constexpr int kJwWaves = 2, kJwMaxE = 16;

__global__ void __launch_bounds__(64 * kJwWaves) k_jw_norms(double *X, int n, int m, unsigned long long *ctl,
                                                           int slot) {
  const int lane = threadIdx.x & 63, i = blockIdx.x * kJwWaves + (threadIdx.x >> 6);
  if (blockIdx.x == 0 && threadIdx.x == 0) {
    ctl[slot ^ 1] = 0ull;
    ctl[2 + (slot ^ 1)] = 0ull;
  }
  if (i >= n) return;
  const double *x = X + (int64_t)i * m;
  double s2 = 0.0;
  for (int l = lane; l < m; l += 64) s2 += x[l] * x[l];
  s2 = wave_sum(s2);
  if (lane == 0) {
    X[(int64_t)n * m + i] = s2;
    atomicMax(&ctl[slot], (unsigned long long)__double_as_longlong(s2));
  }
}

__global__ void __launch_bounds__(64 * kJwWaves) k_jw_round(double *X, int n, int m, int rd,
                                                           unsigned long long *ctl, int slot) {
  const int lane = threadIdx.x & 63, k = blockIdx.x * kJwWaves + (threadIdx.x >> 6);
  const int np = n + (n & 1);
  if (k >= np / 2) return;
  int i, j;
  if (k == 0) {
    i = np - 1;
    j = rd;
  } else {
    i = (rd + k) % (np - 1);
    j = (rd - k + np - 1) % (np - 1);
  }
  if (i >= n || j >= n) return;
  // every load of the pair issued at once (vectors of at most 64 kJwMaxE)
  double *sig = X + (int64_t)n * m;
  double *xi = X + (int64_t)i * m, *xj = X + (int64_t)j * m;
  double u[kJwMaxE], v[kJwMaxE];
#pragma unroll
  for (int e = 0; e < kJwMaxE; ++e) {
    const int l = lane + 64 * e;
    u[e] = l < m ? xi[l] : 0.0;
    v[e] = l < m ? xj[l] : 0.0;
  }
  const double amax = __longlong_as_double((long long)ctl[slot]);
  const double al = sig[i], be = sig[j];
  const double tiny = amax * 1e-28;
  const double tol = fmax(1e-15, 2.3e-16 * sqrt((double)m));
  if (al <= tiny || be <= tiny) return;
  double ga = 0.0;
#pragma unroll
  for (int e = 0; e < kJwMaxE; ++e)
    if (lane + 64 * e < m) ga += u[e] * v[e];
  ga = wave_sum(ga);
  if (fabs(ga) <= tol * sqrt(al * be)) return;
  const bool big = ga * ga > kBig2 * (al * be);
  double c, s;
  const double tn = jacobi_angle(al, be, ga, c, s);
#pragma unroll
  for (int e = 0; e < kJwMaxE; ++e) {
    const int l = lane + 64 * e;
    if (l < m) {
      xi[l] = c * u[e] - s * v[e];
      xj[l] = s * u[e] + c * v[e];
    }
  }
  if (lane == 0) {
    sig[i] = fmax(al - tn * ga, 0.0);
    sig[j] = be + tn * ga;
    atomicOr(&ctl[2 + slot], big ? 3ull : 1ull);
  }
}

// The same sweeps by blocks of columns: the n vectors form nb blocks of
// kJbCols (the last one padded with zero vectors, which never rotate), and a
// round of the round-robin ordering over the blocks pairs them up, one
// workgroup per block pair.  The workgroup holds its 2 kJbCols vectors in LDS
// and rotates every pair among them once (a round-robin over the 16 vectors
// in 15 inner rounds of 8 disjoint pairs, one wave per pair).  Every pair of
// vectors meets at least once per sweep (the pairs inside a block at each of
// its meetings), so the sweep is a block cyclic Jacobi sweep, in nb - 1
// launches instead of n - 1.  Angles, norm updates and the control words are
// those of k_jw_round.
constexpr int kJbCols = 8, kJbThreads = 512;

__global__ void __launch_bounds__(kJbThreads) k_jwb_round(double *X, int n, int m, int nb, int rd,
                                                          unsigned long long *ctl, int slot) {
  extern __shared__ __align__(16) double v[];   // [2 kJbCols][m]
  __shared__ double s_n[2 * kJbCols];
  const int nbp = nb + (nb & 1), k = blockIdx.x;
  int I, J;
  if (k == 0) {
    I = nbp - 1;
    J = rd;
  } else {
    I = (rd + k) % (nbp - 1);
    J = (rd - k + nbp - 1) % (nbp - 1);
  }
  // with an odd block count one block meets the empty block nb (its vectors
  // read as zero and are never written): its own pairs are still rotated
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  constexpr int NW = kJbThreads / 64, NV = 2 * kJbCols;
  double *sig = X + (int64_t)n * m;
  for (int q = wave; q < NV; q += NW) {
    const int c = (q < kJbCols ? I : J) * kJbCols + (q % kJbCols);
    for (int l = lane; l < m; l += 64) v[q * m + l] = c < n ? X[(int64_t)c * m + l] : 0.0;
    if (lane == 0) s_n[q] = c < n ? sig[c] : 0.0;
  }
  __syncthreads();
  const double tiny = __longlong_as_double((long long)ctl[slot]) * 1e-28;
  const double tol = fmax(1e-15, 2.3e-16 * sqrt((double)m));
  int rotated = 0, big = 0;
  for (int r = 0; r < NV - 1; ++r) {
    int a, b;
    if (wave == 0) {
      a = NV - 1;
      b = r;
    } else {
      a = (r + wave) % (NV - 1);
      b = (r - wave + NV - 1) % (NV - 1);
    }
    const double al = s_n[a], be = s_n[b];
    if (al > tiny && be > tiny) {
      // the pair's components in registers (at most kJwMaxE per lane), the
      // sum over the wave by DPP within rows of 16 lanes
      double *xa = v + a * m, *xb = v + b * m;
      double u[kJwMaxE], w[kJwMaxE];
#pragma unroll
      for (int e = 0; e < kJwMaxE; ++e) {
        const int l = lane + 64 * e;
        u[e] = l < m ? xa[l] : 0.0;
        w[e] = l < m ? xb[l] : 0.0;
      }
      double ga = 0.0;
#pragma unroll
      for (int e = 0; e < kJwMaxE; ++e) ga = fma(u[e], w[e], ga);
      ga = group_sum(ga, 64);
      if (fabs(ga) > tol * sqrt(al * be)) {
        big |= ga * ga > kBig2 * (al * be) ? 1 : 0;
        double c, s;
        const double tn = jacobi_angle(al, be, ga, c, s);
#pragma unroll
        for (int e = 0; e < kJwMaxE; ++e) {
          const int l = lane + 64 * e;
          if (l < m) {
            xa[l] = c * u[e] - s * w[e];
            xb[l] = s * u[e] + c * w[e];
          }
        }
        if (lane == 0) {
          s_n[a] = fmax(al - tn * ga, 0.0);
          s_n[b] = be + tn * ga;
        }
        rotated = 1;
      }
    }
    __syncthreads();
  }
  for (int q = wave; q < NV; q += NW) {
    const int c = (q < kJbCols ? I : J) * kJbCols + (q % kJbCols);
    if (c >= n) continue;
    for (int l = lane; l < m; l += 64) X[(int64_t)c * m + l] = v[q * m + l];
    if (lane == 0) sig[c] = s_n[q];
  }
  if (lane == 0 && rotated) atomicOr(&ctl[2 + slot], big ? 3ull : 1ull);
}

template <int E>
void set_lds_cap() {
  (void)hipFuncSetAttribute(reinterpret_cast<const void *>(&k_jacobi<E>),
                            hipFuncAttributeMaxDynamicSharedMemorySize, kJacobiLdsBytes);
}

template <int E>
void launch_e(const Blk *blk, const int *idx, int nblk, int threads, int lds_bytes, double *scratch,
              int max_sweeps, int *sweeps_out, hipStream_t st) {
  hipLaunchKernelGGL(k_jacobi<E>, dim3(nblk), dim3(threads), lds_bytes, st, blk, idx, scratch, max_sweeps,
                     sweeps_out);
}

}  // namespace

void launch_jacobi(const Blk *blk, const int *idx, int nblk, int kind, int threads, int lds_bytes,
                   double *scratch, int max_sweeps, int *sweeps_out, hipStream_t st) {
  if (nblk == 0) return;
  // once per process (thread-safe initialisation of a function-local static)
  static const bool attr_set = [] {
    set_lds_cap<4>();
    set_lds_cap<8>();
    set_lds_cap<12>();
    set_lds_cap<16>();
    set_lds_cap<20>();
    set_lds_cap<24>();
    return true;
  }();
  (void)attr_set;
  switch (kind) {
    case 0: launch_e<4>(blk, idx, nblk, threads, lds_bytes, scratch, max_sweeps, sweeps_out, st); break;
    case 1: launch_e<8>(blk, idx, nblk, threads, lds_bytes, scratch, max_sweeps, sweeps_out, st); break;
    case 2: launch_e<12>(blk, idx, nblk, threads, lds_bytes, scratch, max_sweeps, sweeps_out, st); break;
    case 3: launch_e<16>(blk, idx, nblk, threads, lds_bytes, scratch, max_sweeps, sweeps_out, st); break;
    case 4: launch_e<20>(blk, idx, nblk, threads, lds_bytes, scratch, max_sweeps, sweeps_out, st); break;
    case 5: launch_e<24>(blk, idx, nblk, threads, lds_bytes, scratch, max_sweeps, sweeps_out, st); break;
    default:
      hipLaunchKernelGGL(k_jacobi_global, dim3(nblk), dim3(1024), 0, st, blk, idx, scratch, max_sweeps,
                         sweeps_out, kJwFull, 0, nullptr);
      break;
  }
}

void launch_jacobi_wide_load(const Blk *blk, const int *idx, double *scratch, unsigned long long *ctl,
                             hipStream_t st) {
  hipLaunchKernelGGL(k_jacobi_global, dim3(1), dim3(1024), 0, st, blk, idx, scratch, 0, nullptr, kJwLoad, 0, ctl);
}

void launch_jacobi_wide_sweep(double *X, int n, int m, unsigned long long *ctl, int slot, hipStream_t st) {
  if (m > 64 * kJwMaxE) throw Error(TNQE_ESHAPE, "chip-wide Jacobi: vectors longer than 1024");
  hipLaunchKernelGGL(k_jw_norms, dim3((n + kJwWaves - 1) / kJwWaves), dim3(64 * kJwWaves), 0, st, X, n, m, ctl,
                     slot);
  const int np = n + (n & 1), pairs = np / 2;
  for (int rd = 0; rd < np - 1; ++rd)
    hipLaunchKernelGGL(k_jw_round, dim3((pairs + kJwWaves - 1) / kJwWaves), dim3(64 * kJwWaves), 0, st, X, n, m,
                       rd, ctl, slot);
}

void prepare_jacobi_wide_sweep_blocked() {
  // once per process (thread-safe initialisation of a function-local static)
  static const bool attr_set = [] {
    TNQE_HIP(hipFuncSetAttribute(reinterpret_cast<const void *>(&k_jwb_round),
                                 hipFuncAttributeMaxDynamicSharedMemorySize, 2 * kJbCols * 1024 * 8));
    return true;
  }();
  (void)attr_set;
}

void launch_jacobi_wide_sweep_blocked(double *X, int n, int m, unsigned long long *ctl, int slot, hipStream_t st) {
  if (m > 1024) throw Error(TNQE_ESHAPE, "chip-wide Jacobi: vectors longer than 1024");
  prepare_jacobi_wide_sweep_blocked();
  hipLaunchKernelGGL(k_jw_norms, dim3((n + kJwWaves - 1) / kJwWaves), dim3(64 * kJwWaves), 0, st, X, n, m, ctl,
                     slot);
  const int nb = (n + kJbCols - 1) / kJbCols, nbp = nb + (nb & 1);
  const size_t lds = (size_t)2 * kJbCols * m * sizeof(double);
  for (int rd = 0; rd < nbp - 1; ++rd)
    hipLaunchKernelGGL(k_jwb_round, dim3(nbp / 2), dim3(kJbThreads), lds, st, X, n, m, nb, rd, ctl, slot);
}

void launch_jacobi_wide_finish(const Blk *blk, const int *idx, double *scratch, int sweeps_done, int *sweeps_out,
                               hipStream_t st) {
  hipLaunchKernelGGL(k_jacobi_global, dim3(1), dim3(1024), 0, st, blk, idx, scratch, 0, sweeps_out, kJwFinish,
                     sweeps_done, nullptr);
}

void launch_svd_factor(const Blk *blk, Units u, double *scratch, hipStream_t st) {
  if (u.total == 0) return;
  hipLaunchKernelGGL(k_svd_factor, dim3(u.total), dim3(256), 0, st, blk, u, scratch);
}

}  // namespace tnqe
