// Internal declarations shared by the host sources and the kernel launchers.
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>
#include <stdexcept>
#include <string>
#include <vector>

#include "../../include/tnqe.h"

namespace tnqe {

struct Error : public std::runtime_error {
  tnqe_status st;
  Error(tnqe_status s, const std::string &m) : std::runtime_error(m), st(s) {}
};

#define TNQE_HIP(call)                                                                 \
  do {                                                                                 \
    hipError_t e_ = (call);                                                            \
    if (e_ != hipSuccess)                                                              \
      throw ::tnqe::Error(TNQE_EHIP, std::string(#call) + ": " + hipGetErrorString(e_)); \
  } while (0)

inline void require(bool ok, tnqe_status st, const std::string &msg) {
  if (!ok) throw Error(st, msg);
}

// particle-number shift of a local state k = n_up + 2 n_dn
__host__ __device__ inline int qk_a(int k) { return k & 1; }
__host__ __device__ inline int qk_b(int k) { return k >> 1; }

// Entry x = (k1 * 4 + k2) * 16 + l1 * 4 + l2 of the two-site gate g4(theta)
// on local states (k1, k2) <- (l1, l2) of sites (p, p+1), from c = cos theta,
// s = sin theta (App. A3): on the four modes (p up, p dn, p+1 up, p+1 dn) the
// gate is mid (g2 (x) g2) mid, g2 the single-particle rotation on a mode pair
// and mid = I2 (x) f2 (x) I2 with f2 the fermionic swap (sign on |11>).  mid
// is a symmetric signed permutation, so the entry is one product of two g2
// entries and two signs (the same arithmetic on the host and the device).
__host__ __device__ inline double gate4_entry(double c, double s, int x) {
  const int kq[4] = {0, 2, 1, 3};   // local state k -> mode-bit index (n_up, n_dn)
  const int I = kq[x >> 6] * 4 + kq[(x >> 4) & 3], J = kq[(x >> 2) & 3] * 4 + kq[x & 3];
  // f2 row q: its one nonzero column and sign
  const int f2c[4] = {0, 2, 1, 3};
  const double f2s[4] = {1.0, 1.0, 1.0, -1.0};
  const int ci = (I & 8) | (f2c[(I >> 1) & 3] << 1) | (I & 1), cj = (J & 8) | (f2c[(J >> 1) & 3] << 1) | (J & 1);
  const double si = f2s[(I >> 1) & 3], sj = f2s[(J >> 1) & 3];
  const double g2[16] = {1, 0, 0, 0, 0, c, -s, 0, 0, s, c, 0, 0, 0, 0, 1};
  const double core = g2[(ci >> 2) * 4 + (cj >> 2)] * g2[(ci & 3) * 4 + (cj & 3)];
  return si * core * sj + 0.0;
}

// -------------------------------------------------------------- gate phase
// One quantum-number block of a two-site matrix (or of a single site for the
// exact centre moves).  Rows and columns are grouped in segments by a local
// index k; seg offsets are prefix sums.
struct Blk {
  int pair;            // which ket
  int R, C, n;         // rows, cols, min(R, C)
  int sa, sb;          // quantum numbers of the block's bond sector
  int rs[5];           // row segment starts (by k), rs[4] = R
  int cs[5];           // column segment starts (by k), cs[4] = C
  int j0;              // first index of the sector in the new bond
  int kept;            // singular vectors kept
  int aux0, aux1;      // old offset / old bond dimension for the centre moves
  int grp, mpad;       // Jacobi: lanes per vector pair, padded LDS row length
  int64_t offT, offU, offB, offS;   // scratch offsets (doubles); U is [n][R], B is [n][C]
  int64_t offW;        // work area for blocks too large for LDS (-1: LDS)
  int fact;            // centre moves: 0 Jacobi SVD, 1 Householder QR
};

// Per-pair ket state shared with the kernels.
struct KetTables {
  double **site;       // [pair * N + p]
  int2 *btab;          // [bond][pair][nslot]: (offset, dim) of each sector
  int *bdim;           // [bond][pair]: total bond dimension
  int npair, N, na, nb, nslot;
  __host__ __device__ int slot(int a, int b) const {
    return (a < 0 || b < 0 || a > na || b > nb) ? -1 : a * (nb + 1) + b;
  }
  __host__ __device__ int2 sec(int bond, int pair, int a, int b) const {
    int s = slot(a, b);
    if (s < 0) return make_int2(0, 0);
    return btab[((int64_t)bond * npair + pair) * nslot + s];
  }
  __host__ __device__ int dim(int bond, int pair) const { return bdim[bond * npair + pair]; }
};

// Work units of the gate-phase kernels.  A launch over a block list runs one
// workgroup per unit (a 64 x 64 output tile of a product, or a chunk of
// kGateChunk elements of a gather or scatter), so a large block is spread over
// many compute units instead of looping in one workgroup.  first[i] is the
// first unit of block i (prefix sums, first[n] = total); the host computes the
// counts with the same functions the kernels use to split a unit index.
constexpr int kGateTile = 64, kGateChunk = 2048;
__host__ __device__ inline int gate_tiles(int M, int N) {
  return M <= 0 || N <= 0 ? 0 : ((M + kGateTile - 1) / kGateTile) * ((N + kGateTile - 1) / kGateTile);
}
__host__ __device__ inline int gate_chunks(int64_t n) { return (int)((n + kGateChunk - 1) / kGateChunk); }
// block of unit x: first[i] <= x < first[i + 1] (blocks without units skipped)
__host__ __device__ inline int find_unit(const int *first, int n, int x) {
  int lo = 0, hi = n;
  while (hi - lo > 1) {
    const int mid = (lo + hi) >> 1;
    if (first[mid] <= x) lo = mid;
    else hi = mid;
  }
  return lo;
}
struct Units {
  const int *first;   // device prefix array [n + 1]
  int n, total;
};
// units per block of the split of a truncated two-site block (new A_a
// columns, then new A_{a+1} rows), counted for all n vectors: the launch is
// shaped before the kept counts are known (units past them do nothing)
__host__ __device__ inline int split_units(const Blk &b) {
  return gate_chunks((int64_t)b.R * b.n) + gate_chunks((int64_t)b.n * b.C);
}
// units of the factor product (the kept vectors times the block), counted
// for all n vectors
__host__ __device__ inline int factor_units(const Blk &b) { return gate_tiles(b.n, b.R >= b.C ? b.C : b.R); }

// two-site products per old middle sector (th[0..nth), units: output tiles),
// then the gate into the blocks of the new middle bond (units: element
// chunks; thidx[pair * nslot + slot]: Theta block; cs[2 pair ..] = cos, sin
// of the pair's angle; gates: room for the 16 x 16 gates [pair][256])
void launch_two_site(const KetTables &kt, int a, const Blk *blk, Units ug, const Blk *th, Units ut,
                     const int *thidx, const double *cs, double *gates, double *scratch, hipStream_t st);
// Jacobi SVD of the blocks idx[0..nblk) of blk: sorted singular values (offS)
// and sorted rotated vectors (U = x / s in the columns case, B = x in the rows
// case).  kind k < kJacobiGlobal selects the register-resident kernel with
// E = 4 (k + 1) vector elements per lane (threads and lds_bytes per
// workgroup); kJacobiGlobal is the global-memory fallback.
constexpr int kJacobiMaxE = 24, kJacobiGlobal = kJacobiMaxE / 4, kJacobiKinds = kJacobiGlobal + 1;
constexpr int jacobi_max_threads(int E) { return E > 20 ? 768 : 1024; }
constexpr int kJacobiLdsBytes = 160 * 1024 - 1024;   // dynamic LDS cap per workgroup
void launch_jacobi(const Blk *blk, const int *idx, int nblk, int kind, int threads, int lds_bytes,
                   double *scratch, int max_sweeps, int *sweeps_out, hipStream_t st);
// The global-memory Jacobi of ONE block (blk[idx[0]], kJacobiGlobal storage)
// with its sweeps spread over the chip: load fills the work area and clears
// the four control words ctl; each sweep (slot = sweep & 1) is one norm
// launch and one launch per round, after which bit 0 of ctl[2 + slot] tells
// whether a pair rotated and bit 1 whether one was not yet orthogonal to
// 1e-10 (the sweeps stop at the first sweep without such a rotation); finish
// writes the sorted values and vectors exactly as
// launch_jacobi does (same bits), sweeps_out[idx[0]] = sweeps_done if given.
constexpr int kJwFull = 0, kJwLoad = 1, kJwFinish = 2;
void launch_jacobi_wide_load(const Blk *blk, const int *idx, double *scratch, unsigned long long *ctl,
                             hipStream_t st);
void launch_jacobi_wide_sweep(double *X, int n, int m, unsigned long long *ctl, int slot, hipStream_t st);
// the same sweep by blocks of 8 columns (one launch per round of block pairs;
// not the same bits as the column-pair rounds); prepare_... sets the kernel's
// LDS limit once, so that a stream capture of the launches holds launches only
void prepare_jacobi_wide_sweep_blocked();
void launch_jacobi_wide_sweep_blocked(double *X, int n, int m, unsigned long long *ctl, int slot, hipStream_t st);
void launch_jacobi_wide_finish(const Blk *blk, const int *idx, double *scratch, int sweeps_done, int *sweeps_out,
                               hipStream_t st);
// the other factor of the first `kept` sorted vectors of every block (units:
// factor_units)
void launch_svd_factor(const Blk *blk, Units u, double *scratch, hipStream_t st);
// Truncation of every ket of a gate step on the device (one workgroup per
// ket, whose maxv or fewer singular values are staged in LDS): kept counts
// and offsets into blk, the sector table of `bond` into kt, kept counts into
// kept_out[block] and (keep, discarded weight, gap) into stats[3 ket ..].
constexpr int kSelectLdsBytes = 150 * 1024;
inline size_t select_lds_bytes(int maxv, int nslot) {
  return (size_t)maxv * sizeof(double) + (3 * (size_t)nslot + 1) * sizeof(int);
}
// With scale non-null, scale[ket] receives sqrt(total / kept) of the squared
// singular values (1 when nothing was cut): the renormalisation factor.
void launch_select(Blk *blk, const int *kfirst, int nket, int maxv, const double *scratch, int chi, double tau,
                   const KetTables &kt, int bond, int *kept_out, double *stats, double *scale, hipStream_t st);
// units: split_units; the new A_{a+1} rows of ket t are multiplied by
// scale[t] (scale may be null)
void launch_split_gate(const KetTables &kt, int a, const Blk *blk, Units u, const double *scratch,
                       const double *scale, hipStream_t st);
// units: gate_chunks(R C)
void launch_gather_lq(const KetTables &kt, int q, const Blk *blk, Units u, double *scratch,
                      hipStream_t st);
// units: gate_chunks(n C) for the new A_q rows, then for k = 0..3 the tiles
// gate_tiles(d_k, n) of the left neighbour's product, d_k the dimension of
// the bond q-1 sector that feeds the block through local state k
void launch_apply_lq(const KetTables &kt, int q, const Blk *blk, Units u, const double *scratch,
                     double *const *old_left, hipStream_t st);
// Exact centre moves by Householder QR of the gathered blocks idx[0..nblk)
// of blk (one workgroup each, the block in LDS: qr_lds_bytes(b) <= kQrLdsBytes):
// left = true factorises T^T (LQ of T, a move to the left), else T, with a
// non-negative diagonal of the triangular factor.  Writes
// U [n][R], B [n][C] and S [n] = 1 in the slots the SVD route fills for the
// apply kernels (U takes L, B takes Q for a left move; U takes Q, B takes R
// for a right move), so the move kernels apply L (or R) and write Q unscaled.
constexpr int kQrLdsBytes = 150 * 1024;
inline size_t qr_lds_bytes(const Blk &b) {
  return ((size_t)b.R * b.C + 2 * (size_t)(b.R < b.C ? b.R : b.C)) * sizeof(double);
}
void launch_qr_blocks(const Blk *blk, const int *idx, int nblk, int lds_bytes, bool left, double *scratch,
                      hipStream_t st);
void launch_gather_qr(const KetTables &kt, int p, const Blk *blk, int nblk, double *scratch,
                      hipStream_t st);
void launch_apply_qr(const KetTables &kt, int p, const Blk *blk, int nblk, const double *scratch,
                     double *const *old_right, hipStream_t st);
// zero the entries of site x outside its quantum-number blocks, every ket of
// the set (max_elems: the largest site size of the set, for the grid)
void launch_mask_site(const KetTables &kt, int x, int max_elems, hipStream_t st);
void launch_copy(double *const *dst, double *const *src, const int64_t *count, int n,
                 hipStream_t st);
void launch_site_sign(double *const *site, const int *rows, int n, int cols, hipStream_t st);

// -------------------------------------------------------------- environment sweep
// Sector tables of the items (bra MPS and rotated kets) and the bra/ket item
// of every pair in a launch.
struct EnvGeom {
  const int2 *tab;     // [item][bond][slot]: (offset, dim) of the sector in the bond
  const int *D;        // [item][bond]: bond dimension
  const int *bra;      // [pair] bra item
  const int *ket;      // [pair] ket item
  int nbond, nslot;
  __host__ __device__ int2 sec(int item, int b, int s) const {
    return s < 0 ? make_int2(0, 0) : tab[((int64_t)item * nbond + b) * nslot + s];
  }
  __host__ __device__ int dim(int item, int b) const { return D[item * nbond + b]; }
};

// One entry of a launch's work list: problem `desc` of the site's list for
// pair `pair` of the batch, whose workgroups (output tiles, or 256-item
// chunks, of that pair's own extents) start at workgroup `first`.  Entries
// are in increasing `first`; problems with empty extents have no entry.
struct EnvWork {
  int desc, pair, first;
};

// X[(c, s, k)] = L[(c, s)] x ket site x block (s, k, sk); bra sector sbra = s + shift(c)
struct EnvG1 {
  int x, nw, sbra, s, k, sk;
  int64_t offL, offX;
};
// L_{x+1}[(c, s)] = sum_q bra site x block (sa[q], kp[q], sbn)^T Y[offY[q]]
struct EnvG2 {
  int x, nw, sbn, s, nseg;
  int sa[4], kp[4];
  int64_t offY[4], offL;
};
// dense coupling: Y[a][r0..r0+nr][b] += f W[nr][nc] X[a][c0..c0+nc][b], one
// batch per bra row a of the block (bra sector sa at bond x, ket sector s at x+1)
struct EnvGD {
  int x, sa, s, nr, nc, r0, c0, nw_in, nw_out;
  int64_t offY, offX, valoff;
  double f;
};
// one (bra sector, local state) term of the final element
struct EnvFinal {
  int sa, kp;
  int64_t offY;
};

// tileM x tileN output tiles; work[0..nwork) covers nwg workgroups.  cm
// (FP32 storage only) selects the matrix-core arithmetic: 0 FP32, 1 BF16
// operands, 2 split BF16 (hi hi + hi lo + lo hi); FP32 accumulation.
template <typename T>
void launch_env_g1(const EnvG1 *d, const EnvWork *work, int nwork, int nwg, int tileM, int tileN,
                   const EnvGeom &g, const T *const *L, const T *const *ket, T *const *X, hipStream_t st,
                   int cm = 0);
template <typename T>
void launch_env_g2(const EnvG2 *d, const EnvWork *work, int nwork, int nwg, int tileM, int tileN,
                   const EnvGeom &g, const T *const *bra, const T *const *Y, T *const *Ln, hipStream_t st,
                   int cm = 0);
template <typename T>
void launch_env_gd(const EnvGD *d, const EnvWork *work, int nwork, int nwg, int tileM, int tileN,
                   const EnvGeom &g, const T *const *vals, const T *const *X, T *const *Y, hipStream_t st,
                   int cm = 0);

// channel mix: Y[c', s, k'] = sum over sources of coef * X[c, s_in, k].
// One source of a task: a sparse MPO group (CSR over output x input channel,
// kept on the device once per structure) applied to one X block:
// Y[a][w'][b] += factor sum_z vals[vbase + z] X[offX + (a nw_in + col[cp + z]) db + b]
// for z in [rowptr[rp + w'], rowptr[rp + w' + 1]).
struct MixSrc {
  int64_t offX;        // X block [da][nw_in][db]
  int64_t vbase;       // value index of the group's first nonzero
  int64_t rp, cp;      // offsets of the group's row pointers and column indices
  int nw_in;
  int group;           // host bookkeeping: index into the site's MPO groups
  double factor;       // local-operator matrix element
};
struct MixTask {
  int64_t offY;        // Y block [da][nw_out][db], da = dim_bra(x, sa), db = dim_ket(x + 1, s)
  int x, sa, s, nw_out;
  int src0, nsrc;      // range in the site's source array
};
// A channel-mix thread computes kMixCols ket columns of kMixRows bra rows
// (same output channel): the coupling structure is loaded once for them.
constexpr int kMixRows = 8;
constexpr int kMixCols = 1;
constexpr int kMixUnroll = 2;
// The vector channel mix (blocks with an even number db of ket columns): a
// thread computes the column pair (2t, 2t + 1) of kMix2Rows bra rows.
constexpr int kMix2Rows = 4;
struct MixArgs {
  const MixTask *tasks;
  const EnvWork *work;      // (task, pair, first chunk of 256 items)
  int nwork, nchunk;
  const MixSrc *srcs;
  const int *rowptr, *col;  // CSR structure of the MPO groups
  const double *vals;       // [basis][nnz of all sites]
  int64_t basis_stride;
  const int *basis;         // [pair]
};
template <typename T>
void launch_mix(const MixArgs &a, const EnvGeom &g, const T *const *X, T *const *Y, hipStream_t st);
// the same for the task-pairs of even db, column pairs loaded as one vector
// (X and Y offsets even, every pair's buffers 16-byte aligned)
template <typename T>
void launch_mix2(const MixArgs &a, const EnvGeom &g, const T *const *X, T *const *Y, hipStream_t st);

template <typename T>
void launch_env_init(T *const *L, int npair, int64_t size, hipStream_t st);

// final element at the last site x: out[pair][w] = sum_{a', k'} bra[a', k', 0] Y[k'][a'][w][0], compensated
template <typename T>
void launch_env_final(const EnvGeom &g, int x, const double *const *bra, const T *const *Y, const EnvFinal *fin,
                      int nk, int nw, double *out, int npair, hipStream_t st);

// MPO coefficients of every basis moved along a fixed direction:
// y[b][j] = x[b][j] + a z[j], b < nbasis, j < nnz
void launch_shift_vals(const double *x, const double *z, double a, int64_t nnz, int nbasis, double *y,
                       hipStream_t st);
// FP32 copies of FP64 arrays
void launch_cast(const double *const *src, float *const *dst, const int64_t *count, int n, hipStream_t st);

// -------------------------------------------------------------- expanded one-hot pencil
// One FP64 matrix-core GEMM C (M x N) = sum_k A(m, k) B(k, n) of the dense
// contractions of the one-hot pencil: left and right environment steps with a
// dense MPO site W[w_in][w_out][k'][k], the two-site blocks, and the dense
// one-hot matrix.  kind selects how (m, k, n) map to the operands' layouts
// (d0..d2 are the extra dimensions those maps need):
//   Plain    A[m K + k]       B[k N + n]        C[m N + n]
//   PlainBT  A[m K + k]       B[n K + k]        C[m N + n]
//   PlainAT  A[k M + m]       B[k N + n]        C[m N + n]
//   WX       m = (wo, ko), k = (wi, ki): A = W[((wi d0 + wo) 4 + ko) 4 + ki],
//            n = (a, x < d2): B[((wi d1 + a) 4 + ki) d2 + x]            C[m N + n]
//   BraL     A[k M + m], k = (a, k'), n = (w, b < d1): B[((w 4 + k') d0 + a) d1 + b],
//            C[((w M) + m) d1 + b]
//   RX2      A = W[((w d0 + w') 4 + k') 4 + k], m = (w, k'), k = (w', k):
//            B[(w' N + n) 4 + k]                                        C[m N + n]
//   BraR     A[m K + k], n = (w, a < d0): B[(w K + k) d0 + a]           C[((w M) + m) d0 + a]
//   A3       A as WX; n = (kp, l < d1, b < d2), k = (w1, kq2):
//            B[(w1 4 + kp) (4 d1 d2) + (l 4 + kq2) d2 + b]              C[m N + n]
//   A4       m = (l, kp, kq), k = (w2, b < d1):
//            A[(w2 4 + kq) (4 d0 d1) + (kp d0 + l) d1 + b], B[(w2 d2 + n) d1 + b], C[m N + n]
//   D1       m = (w, kpkp2), k = w1: A[(w d0 + k) 16 + kpkp2]; B[k N + n]; C[m N + n]
//   D3       m = ((l d0 + l2) 16 + kpkp2) 16 + kqkq2, k = w2:
//            A[(l d0 + l2) (256 d1) + (kpkp2 d1 + k) 16 + kqkq2]; B[k N + n],
//            n = (r, r2 < d2); stored to C[map(l, kp, kq, r) n_oh + map(l2, kp2, kq2, r2)]
//            when both one-hot numbers exist (map: dense T index -> one-hot number or -1)
enum OhKind { kOhPlain, kOhPlainBT, kOhPlainAT, kOhWX, kOhBraL, kOhRX2, kOhBraR, kOhA3, kOhA4, kOhD1, kOhD3 };
struct OhGemm {
  int kind, M, N, K;
  const double *A, *B;
  double *C;
  int d0, d1, d2;
  const int *map;
  int n_oh;
};
void launch_oh_gemm(const OhGemm &g, hipStream_t st);
// out[m ld + col] = V[idx[m]] (+ f S[idx[m]] when S is not null), m < n
void launch_oh_gather(const double *V, const double *S, double f, const int *idx, int n, double *out, int ld, int col,
                      hipStream_t st);
// diagonal overlap block from the overlap environments and the one-hot
// tuples oh[m] = (l, kp, kq, r): Sd[m][n] = [kp, kq equal] LS[l][l2] RS[r][r2]
// (LS [Db][Db], RS [Db2][Db2]); Hd += e_core Sd
void launch_oh_sd(const int4 *oh, int n, const double *LS, int Db, const double *RS, int Db2, double e_core,
                  double *Sd, double *Hd, hipStream_t st);

// ------------------------------------------------- generalized-sweep step
// expanded pencil (H', S') [D][D] in the combined order (code: see kernel)
void launch_sw_assemble(const int *code, int D, int n, int M, const double *H, const double *S, const double *Hd,
                        const double *Sd, const double *Hc, const double *Sc, double *Hx, double *Sx, hipStream_t st);
// keep[j] for the columns of S taken in order (A: a copy of S, overwritten)
void launch_sw_discard(double *A, const double *S, int D, double tol, int *keep, hipStream_t st);
void launch_sw_gather(const double *Hx, const double *Sx, int D, const int *kidx, int Dk, double *Hk, double *Sk,
                      hipStream_t st);
void launch_sw_whiten(const double *U, const double *lam, int Dk, int r, double *X, hipStream_t st);
void launch_sw_shift(const double *C, int r, double *B, double *out, hipStream_t st);
void launch_sw_update(const double *ck, const int *col, const double *told, int told_ld, int n, const int *dense_of,
                      double *T, int64_t tsize, double *tnew, double *stats, hipStream_t st);
void launch_sw_gate_blocks(const Blk *blk, int nblk, const double *gates, const double *T, int Dq, const int *offp,
                           const int *offq, int na, int nb1, double *scratch, hipStream_t st);
// single-site mitigation: the gate in the one-hot basis [n][n]; the two-site
// coefficients of A_p A_{p+1} at the one-hot entries; their dense scatter
void launch_sw_onehot_gate(const int4 *oh, const int *map, int n, int Dq, const double *G16, double *Gm,
                           hipStream_t st);
void launch_sw_product(const double *Ap, const double *Aq, int Dn, int Dq, const int4 *oh, int n, double *x,
                       hipStream_t st);
void launch_sw_scatter(const double *x, int n, const int *dense_of, double *T, int64_t tsize, hipStream_t st);
constexpr int kXiMaxValues = 8192;   // singular values per gate in k_sw_xi (LDS)
void launch_sw_xi(const Blk *blk, const int *first, int ngate, int max_values, const double *scratch, int chi,
                  double *xi, hipStream_t st);

// -------------------------------------------------------------- eigensolve
// For each subspace s: H, S at offs[s] ([M_s][M_s] row-major); writes
// out[s * (8 + kMaxM) + ...] = E, cond_S, lambda_min, n_dropped, kappa1, status, -, -, c[0..M_s).
constexpr int kMaxM = 32;
void launch_gep(const double *H, const double *S, const int *Ms, const int64_t *offs, int nsub,
                double eps_S, double *out, hipStream_t st);

}  // namespace tnqe
