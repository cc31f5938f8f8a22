// Step (c), Eq. (5): C = V Lambda V^{t*} by parallel cyclic Jacobi in FP64, one workgroup.
//
// A sweep is m-1 rounds (m = n rounded up to even; an odd n gets a zero row and
// column, which never rotates) of m/2 disjoint 2x2 Hermitian rotations, in
// round-robin order: every index pair meets once per sweep.  For a pair (p, q) with
// a = A[p][p], b = A[q][q], beta = A[p][q], g = b - a:
//   D = sqrt(g^2 + 4 |beta|^2),  den = sqrt(2 D (D + |g|)),
//   c = (D + |g|) / den,  J[p][q] = sgn(g) 2 beta / den,  J[q][p] = -conj(J[p][q]),
//   J[p][p] = J[q][q] = c,   A <- J^H A J,   V <- V J,
// which zeroes A[p][q] and moves t|beta| = sgn(g) 2 |beta|^2 / (D + |g|) from A[p][p]
// to A[q][q] (the textbook t = sgn(theta)/(|theta| + sqrt(1 + theta^2)),
// theta = g / (2|beta|), rewritten to need two square roots and one division).
//
// Layout.  A is kept in slot coordinates: pair k of every round sits on slots 2k and
// 2k+1, and between rounds the indices move through the slots by one fixed
// permutation (the circle method: one index stays, the others advance one place),
// so the A addresses a thread touches are the same in every round.  The diagonal
// lives in the rotation data (a rotation knows its pair's new diagonal entries); the
// off-diagonal entries live in two buffers that share one [NMAX][NMAX+1] array (the
// upper and the lower triangle).  A round reads one buffer and writes the other,
// already permuted for the next round, so it needs a single barrier:
//   wave 0, lane k: the next round's rotation of pair k, from this round's data: its
//     off-diagonal entry is one output of this round's 2x2 block rotation, recomputed
//     here, and its diagonal entries are in this round's rotation data;
//   the block waves: A <- J^H A J on the 2x2 blocks {2P, 2P+1} x {2Q, 2Q+1}, one
//     column of a block per task (a pair's own block: its off-diagonal entry, which
//     becomes zero if the pair rotates);
//   the other waves: V <- V J in place, one (row, pair) per task; V's columns stay in
//     index order, so a task looks up the two indices on its pair's slots.
// Square roots and reciprocals use hardware seeds refined by Newton steps.  C is
// scaled by an exact power of two so that its Frobenius norm is O(1).  A rotation is
// skipped when |beta| <= 1e-15 sqrt(|a b|) or |beta| <= 1e-16 ||C||_F (about the unit
// roundoff times ||C||: such an entry is within the rounding already made in forming C
// and in every rotation); the iteration stops at the start of a sweep when every
// off-diagonal entry passes that test.  The
// result is sorted by decreasing eigenvalue and each eigenvector's phase is fixed.
#include <type_traits>

#include "hh_internal.h"

namespace hh {
namespace {

constexpr double kRelTol = 1e-15;
constexpr double kAbsTol = 1e-16;
// Workgroup per size class: wave 0 computes the rotations, kBlockWaves waves rotate
// A's blocks, the others rotate V.  n <= 32: 13 waves, one task per lane (a round is
// latency-bound); n <= 64: 16 waves, the most a workgroup holds (four block tasks and
// three V tasks per lane).
template <int NMAX>
struct JacobiShape;
template <>
struct JacobiShape<32> {
  static constexpr int kThreads = 832, kBlockWaves = 4;
};
template <>
struct JacobiShape<64> {
  static constexpr int kThreads = 1024, kBlockWaves = 4;
};
template <int NMAX>
constexpr int threads_for() { return JacobiShape<NMAX>::kThreads; }
constexpr size_t kCuLdsBytes = 160 * 1024;

__device__ __forceinline__ double2 zmul(double2 a, double2 b) {
  return make_double2(a.x * b.x - a.y * b.y, a.x * b.y + a.y * b.x);
}
__device__ __forceinline__ double2 zconj(double2 a) { return make_double2(a.x, -a.y); }
__device__ __forceinline__ double2 zscale(double2 a, double s) { return make_double2(a.x * s, a.y * s); }
__device__ __forceinline__ double2 zadd(double2 a, double2 b) { return make_double2(a.x + b.x, a.y + b.y); }
__device__ __forceinline__ double2 zsub(double2 a, double2 b) { return make_double2(a.x - b.x, a.y - b.y); }

// 1/sqrt(x) and 1/x for x > 0: hardware seeds refined by two Newton steps each
// (quadratic convergence to double precision).
__device__ __forceinline__ double rsq64(double x) {
  double y = __builtin_amdgcn_rsq(x);
  const double hx = 0.5 * x;
  y = y * fma(-hx * y, y, 1.5);
  y = y * fma(-hx * y, y, 1.5);
  return y;
}
__device__ __forceinline__ double rcp64(double x) {
  double y = __builtin_amdgcn_rcp(x);
  y = y * fma(-x, y, 2.0);
  y = y * fma(-x, y, 2.0);
  return y;
}

// Per-round rotation data, indexed by slot: the pair on slots p = 2k, q = 2k+1 has
// cd[p] = (c, new A[p][p]), cd[q] = (c, new A[q][q]), e[q] = J[p][q], e[p] = J[q][p].
// A pair rotates iff e[q] is nonzero (a rotating pair has |beta| > 1e-16 ||C||_F after
// scaling, so J[p][q] cannot underflow to zero); a pair that does not rotate has c = 1,
// e = 0 and its diagonal entries as they are.
template <int NMAX>
struct RoundParams {
  double2 cd[NMAX];
  double2 e[NMAX];
};

// Circle-method schedule on m slots: slot 2k is place k and slot 2k+1 place m-1-k, so
// the pairs (place k, place m-1-k) are the slot pairs (2k, 2k+1).  After a round the
// index in place 0 stays and every other index advances one place (m-1 wraps to 1):
// every two indices share a pair once in m-1 rounds, after which each index is back on
// its own slot.
__device__ __forceinline__ int slot_place(int s, int m) { return (s & 1) ? m - 1 - (s >> 1) : s >> 1; }
__device__ __forceinline__ int place_slot(int p, int m) { return 2 * p < m ? 2 * p : 2 * (m - 1 - p) + 1; }
// the slot that the entry on slot s moves to after a round, and the one it came from
__device__ __forceinline__ int slot_after(int s, int m) {
  const int p = slot_place(s, m);
  return place_slot(p == 0 ? 0 : (p == m - 1 ? 1 : p + 1), m);
}
__device__ __forceinline__ int slot_before(int s, int m) {
  const int p = slot_place(s, m);
  return place_slot(p == 0 ? 0 : (p == 1 ? m - 1 : p - 1), m);
}
// the matrix index on slot s in round r of a sweep (0 <= r < m - 1)
__device__ __forceinline__ int slot_index(int s, int r, int m) {
  const int p = slot_place(s, m);
  if (p == 0) return 0;
  int t = p - 1 - r;
  if (t < 0) t += m - 1;
  return place_slot(t + 1, m);
}

// Rotation of the pair on slots 2k, 2k+1 from its diagonal entries a, b and its
// off-diagonal entry beta.
template <int NMAX>
__device__ __forceinline__ void set_rotation(RoundParams<NMAX> &P, int k, double a, double b, double2 beta,
                                             double abs2) {
  // computed whether or not the pair rotates, then selected (no branch around the
  // arithmetic)
  const double ab2 = beta.x * beta.x + beta.y * beta.y;
  const bool rot = ab2 > kRelTol * kRelTol * fabs(a * b) && ab2 > abs2;
  const double g = b - a, ag = fabs(g), sg = g >= 0.0 ? 1.0 : -1.0;
  const double w = g * g + 4.0 * ab2;
  const double D = w * rsq64(w);
  const double inv = rsq64(2.0 * D * (D + ag));  // 1 / den
  const double tab = sg * 2.0 * ab2 * rcp64(D + ag);
  const double c = rot ? (D + ag) * inv : 1.0;
  const double2 eq = rot ? make_double2(sg * 2.0 * inv * beta.x, sg * 2.0 * inv * beta.y)  // J[p][q]
                         : make_double2(0.0, 0.0);
  P.cd[2 * k] = make_double2(c, rot ? a - tab : a);
  P.cd[2 * k + 1] = make_double2(c, rot ? b + tab : b);
  P.e[2 * k + 1] = eq;
  P.e[2 * k] = rot ? make_double2(-eq.x, eq.y) : make_double2(0.0, 0.0);  // J[q][p] = -conj(J[p][q])
}

// Off-diagonal entries in slot coordinates: buffer 0 keeps entry (x, y), x < y, at
// [x][y], buffer 1 keeps the same value at [y][x].  Address of (x, y), x < y, in buffer b:
template <int LD>
__device__ __forceinline__ int abuf_addr(int b, int x, int y) { return b ? y * LD + x : x * LD + y; }
// Writes entry (u, v), u != v in either order, into buffer b: the value of entry
// (min, max), i.e. val conjugated when u > v.
template <int LD>
__device__ __forceinline__ void abuf_write(double2 *A, int b, int u, int v, double2 val) {
  const int lo = u < v ? u : v, hi = u < v ? v : u;
  A[abuf_addr<LD>(b, lo, hi)] = make_double2(val.x, u < v ? val.y : -val.y);
}

// Column y of J_P^H M J_Q for a 2x2 block M of A (rows 2P, 2P+1 and columns 2Q, 2Q+1
// in slot coordinates), given m0y = M[0][y], m0o = M[0][1-y], m1y = M[1][y],
// m1o = M[1][1-y] and the two rotations' c and J[2P][2P+1] (cP, eP), c and J[2Q][2Q+1]
// (cQ, eQ): entries (2P, 2Q+y) and (2P+1, 2Q+y) of the rotated block.
__device__ __forceinline__ void block_column(double2 m0y, double2 m0o, double2 m1y, double2 m1o, double cP,
                                             double2 eP, double cQ, double2 eQ, int y, double2 &o0,
                                             double2 &o1) {
  const double2 w = y ? eQ : make_double2(-eQ.x, eQ.y);  // J_Q[2Q+1-y][2Q+y]
  const double2 t0 = zadd(zscale(m0y, cQ), zmul(m0o, w));
  const double2 t1 = zadd(zscale(m1y, cQ), zmul(m1o, w));
  o0 = zsub(zscale(t0, cP), zmul(eP, t1));
  o1 = zadd(zmul(zconj(eP), t0), zscale(t1, cP));
}

// C into A (scaled by an exact power of two so that its Frobenius norm is O(1))
// and V = I, both [n][NMAX + 1] in LDS.  C comes from the covariance partials when
// given (the same fixed-order sums as the covariance's own assembly), else from
// cov; the lower triangle and the real diagonal are read, A is Hermitian.
// Returns the scale; red[0] holds ||C||_F * scale on return.
template <int NMAX, int kThreads>
__device__ double load_scaled(const EighProblem &pr, double2 *A, double2 *V, double *red) {
  constexpr int LD = NMAX + 1;
  const int n = pr.n, tid = threadIdx.x;
  const double2 *__restrict__ C = reinterpret_cast<const double2 *>(pr.cov);
  if (pr.part2) {
    const int D = pr.D, G2 = pr.g2;
    const size_t L = partial_len(D);
    double2 *Cw = reinterpret_cast<double2 *>(const_cast<double *>(pr.cov));
    for (int e = tid; e < n * n; e += kThreads) {
      const int s = e / n, t = e - (e / n) * n;
      const int lo = s < t ? s : t, hi = s < t ? t : s;
      double re = 0.0, qst = 0.0, qts = 0.0, mm = 0.0, alo = 0.0, ahi = 0.0, ais = 0.0, ait = 0.0;
      for (int g = 0; g < G2; ++g) {
        const double *q = pr.part2 + g * L;
        re += q[lo * D + hi];
        qst += q[(size_t)D * D + s * D + t];
        qts += q[(size_t)D * D + t * D + s];
        alo += q[2 * D * D + lo];
        ahi += q[2 * D * D + hi];
        ais += q[2 * D * D + D + s];
        ait += q[2 * D * D + D + t];
        mm += q[2 * D * D + 2 * D];
      }
      const double2 c = make_double2((re + mm) + (alo + ahi), (qst - qts) + (ait - ais));
      Cw[e] = c;
      A[s * LD + t] = c;
    }
  } else {
    for (int e = tid; e < n * n; e += kThreads) {
      const int i = e / n, j = e - (e / n) * n;
      A[i * LD + j] = C[e];
    }
  }
  __syncthreads();
  // Frobenius norm -> exact power-of-two scale
  double s2 = 0.0;
  for (int e = tid; e < n * n; e += kThreads) {
    const int i = e / n, j = e - (e / n) * n;
    const double2 v = i > j ? A[i * LD + j] : i < j ? zconj(A[j * LD + i]) : make_double2(A[i * LD + i].x, 0.0);
    s2 += v.x * v.x + v.y * v.y;
  }
  red[tid] = s2;
  __syncthreads();
  if (tid == 0) {
    double t = 0.0;
    for (int k = 0; k < kThreads; ++k) t += red[k];
    red[0] = t;
  }
  __syncthreads();
  const double fro = sqrt(red[0]);
  const double scale = fro > 0.0 ? ldexp(1.0, -ilogb(fro)) : 1.0;

  // Hermitian input: the lower triangle and the real diagonal are read.  Each
  // thread reads the two mirrored entries of its own pair (i > j), so the
  // in-place update needs no extra barrier.
  for (int e = tid; e < n * n; e += kThreads) {
    const int i = e / n, j = e - (e / n) * n;
    if (i > j) {
      const double2 a = zscale(A[i * LD + j], scale);
      A[i * LD + j] = a;
      A[j * LD + i] = zconj(a);
    } else if (i == j) {
      A[i * LD + i] = make_double2(A[i * LD + i].x * scale, 0.0);
    }
    V[i * LD + j] = make_double2(i == j ? 1.0 : 0.0, 0.0);
  }
  __syncthreads();
  if (tid == 0) red[0] = fro * scale;
  __syncthreads();
  return scale;
}

// Sorts by decreasing eigenvalue (ties: lower index first) from A's diagonal and V's
// columns, undoes the scale, fixes each column's phase (the lowest row whose modulus
// is within 1e-12 of the largest becomes real > 0) and writes the outputs.
template <int NMAX>
__device__ void store_sorted(const EighProblem &pr, const double2 *A, const double2 *V, double scale, int *rank_of,
                             int info_value) {
  constexpr int LD = NMAX + 1;
  const int n = pr.n, tid = threadIdx.x;
  double *__restrict__ evals = pr.evals;
  double2 *__restrict__ evecs = reinterpret_cast<double2 *>(pr.evecs);
  if (tid < n) {
    const double di = A[tid * LD + tid].x;
    int rk = 0;
    for (int j = 0; j < n; ++j) {
      const double dj = A[j * LD + j].x;
      rk += (dj > di) || (dj == di && j < tid);
    }
    rank_of[tid] = rk;
    evals[rk] = di / scale;
  }
  __syncthreads();
  if (tid < n) {
    const int k = tid, col = rank_of[k];
    double mx = 0.0;
    for (int j = 0; j < n; ++j) {
      const double2 v = V[j * LD + k];
      mx = fmax(mx, sqrt(v.x * v.x + v.y * v.y));
    }
    int js = 0;
    for (int j = n - 1; j >= 0; --j) {
      const double2 v = V[j * LD + k];
      if (sqrt(v.x * v.x + v.y * v.y) >= mx * (1.0 - 1e-12)) js = j;
    }
    const double2 vs = V[js * LD + k];
    const double ms = sqrt(vs.x * vs.x + vs.y * vs.y);
    const double2 ph = ms > 0.0 ? make_double2(vs.x / ms, -vs.y / ms) : make_double2(1.0, 0.0);
    for (int j = 0; j < n; ++j) {
      const double2 v = (j == js) ? make_double2(ms, 0.0) : zmul(V[j * LD + k], ph);
      evecs[j * n + col] = v;
    }
  }
  if (tid == 0) *pr.info = info_value;
}

template <int NMAX>
__global__ __launch_bounds__(threads_for<NMAX>()) void eigh_jacobi(EighBatch batch, int max_sweeps) {
  constexpr int kThreads = threads_for<NMAX>();
  constexpr int BW = JacobiShape<NMAX>::kBlockWaves;
  // one workgroup per problem of the batch
  const EighProblem &pr = batch.prob[blockIdx.x];
  const int n = pr.n;
  constexpr int LD = NMAX + 1;
  constexpr int NPMAX = NMAX / 2;
  constexpr int TPB = (NPMAX * NPMAX + 64 * BW - 1) / (64 * BW);  // block tasks per lane
  constexpr int VW = kThreads / 64 - 1 - BW;                      // waves rotating V
  constexpr int GPW = 64 / NMAX;                                  // pairs per V wave and item
  constexpr int NG = NPMAX / GPW;                                 // V items
  constexpr int VPT = (NG + VW - 1) / VW;                         // V items per wave
  static_assert(kThreads % 64 == 0 && VW > 0 && NMAX * LD < 65536, "workgroup shape");
  extern __shared__ double2 smem[];
  double2 *const A = smem;              // the two off-diagonal buffers, [NMAX][LD]
  double2 *const V = smem + NMAX * LD;  // [n][LD], columns in index order
  __shared__ RoundParams<NMAX> prm[2];
  __shared__ double dg[NMAX];                       // diagonal in slot order, at the start of a sweep
  __shared__ unsigned short vidx[NMAX - 1][NPMAX];  // indices on pair k's slots in round r: p | q << 8
  __shared__ int flag;
  __shared__ double red[kThreads];
  __shared__ int rank_of[NMAX];
  const int tid = threadIdx.x, lane = tid & 63;
  const int wave = __builtin_amdgcn_readfirstlane(tid >> 6);  // the same for a wave's lanes
  const int m = n + (n & 1);
  const int np = m / 2;

  // Block tasks of waves 1..BW: task t < np is pair t's own block (its off-diagonal
  // entry (2t, 2t+1)), task np + 2b + y column y of the b-th block P < Q.  Precomputed
  // per task: bmeta = x0 | c0 << 8 | conj output 0 << 16 | conj output 1 << 17 | kind << 24
  // (kind 0: none, 1: own block, 2: block column; x0 = 2P, c0 = 2Q + y); bbase = the
  // address of M[0][y] (own block: of its entry) in buffer 0 | in buffer 1 << 16 (the
  // block's other entries are at fixed offsets from it); bw0, bw1 = the addresses of the
  // two outputs after the round's permutation in buffer 0 and 1 (low, high half).
  int bmeta[TPB], bbase[TPB], bw0[TPB], bw1[TPB];
#pragma unroll
  for (int u = 0; u < TPB; ++u) {
    bmeta[u] = bbase[u] = bw0[u] = bw1[u] = 0;
    const int t = (tid - 64) + 64 * BW * u;
    if (wave < 1 || wave > BW || t >= np * np) continue;
    if (t < np) {
      const int x0 = 2 * t, c0 = 2 * t + 1;
      const int w0 = slot_after(x0, m), wc = slot_after(c0, m);
      const int lo = w0 < wc ? w0 : wc, hi = w0 < wc ? wc : w0;
      bbase[u] = abuf_addr<LD>(0, x0, c0) | abuf_addr<LD>(1, x0, c0) << 16;
      bw0[u] = abuf_addr<LD>(0, lo, hi);
      bw1[u] = abuf_addr<LD>(1, lo, hi);
      bmeta[u] = x0 | c0 << 8 | (w0 > wc) << 16 | 1 << 24;
    } else {
      int bi = (t - np) >> 1, P = 0;
      const int y = (t - np) & 1;
      while (bi >= np - 1 - P) {
        bi -= np - 1 - P;
        ++P;
      }
      const int Q = P + 1 + bi;
      const int x0 = 2 * P, c0 = 2 * Q + y;
      const int w0 = slot_after(x0, m), w1 = slot_after(x0 + 1, m), wc = slot_after(c0, m);
      bbase[u] = abuf_addr<LD>(0, x0, c0) | abuf_addr<LD>(1, x0, c0) << 16;
      bw0[u] = abuf_addr<LD>(0, w0 < wc ? w0 : wc, w0 < wc ? wc : w0) |
               abuf_addr<LD>(0, w1 < wc ? w1 : wc, w1 < wc ? wc : w1) << 16;
      bw1[u] = abuf_addr<LD>(1, w0 < wc ? w0 : wc, w0 < wc ? wc : w0) |
               abuf_addr<LD>(1, w1 < wc ? w1 : wc, w1 < wc ? wc : w1) << 16;
      bmeta[u] = x0 | c0 << 8 | (w0 > wc) << 16 | (w1 > wc) << 17 | 2 << 24;
    }
  }

  // Rotation lanes (wave 0, lane k < np): the next round's pair k is on slots rs0, rs1
  // in this round; its off-diagonal entry is row rx of column ry of this round's block
  // (rx0 / 2, rcq / 2), rx0 < rcq, conjugated when rs0's pair is the later one (rconj);
  // rbase as bbase.  For m = 2 the pair is the same in every round (rsame; rbase: the
  // entry (0, 1)).
  int rs0 = 0, rs1 = 0, rx0 = 0, rcq = 0, rbase = 0, rflags = 0;  // rflags: ry | rx << 1 | rconj << 2 | rsame << 3
  if (wave == 0 && lane < np) {
    rs0 = slot_before(2 * lane, m);
    rs1 = slot_before(2 * lane + 1, m);
    const int P0 = rs0 >> 1, P1 = rs1 >> 1;
    const bool rsame = P0 == P1, rconj = P0 > P1;
    const int rP = rconj ? P1 : P0, rQ = rconj ? P0 : P1;
    const int rx = (rconj ? rs1 : rs0) & 1, ry = (rconj ? rs0 : rs1) & 1;
    rx0 = 2 * rP;
    rcq = 2 * rQ;
    const int xa = rsame ? 0 : rx0, ca = rsame ? 1 : rcq + ry;
    rbase = abuf_addr<LD>(0, xa, ca) | abuf_addr<LD>(1, xa, ca) << 16;
    rflags = ry | rx << 1 | rconj << 2 | rsame << 3;
  }

  // V tasks of the other waves: one row per lane, the wave's lanes in groups of NMAX
  // rows that each take one pair, so the rotation data and the indices a group reads
  // are LDS broadcasts.  Item g of a wave is the pairs GPW g .. GPW g + GPW - 1.
  const int vl = tid - 64 * (1 + BW);
  const int vrow = (vl & 63) % NMAX, vsub = (vl & 63) / NMAX, vwave = vl >> 6;

  const double scale = load_scaled<NMAX, kThreads>(pr, A, V, red);
  const double fro = red[0] / scale;  // Frobenius norm of C (exactly, scale is a power of two)
  const double abs2 = (kAbsTol * fro * scale) * (kAbsTol * fro * scale);
  // the diagonal out of A; the zero row and column of an odd n (buffer 0 and V); the
  // index table of the V tasks
  if (tid < NMAX) dg[tid] = tid < n ? A[tid * LD + tid].x : 0.0;
  if (m > n) {
    for (int i = tid; i < n; i += kThreads) {
      A[i * LD + n] = make_double2(0.0, 0.0);
      V[i * LD + n] = make_double2(0.0, 0.0);
    }
  }
  for (int e = tid; e < (m - 1) * np; e += kThreads) {
    const int r = e / np, k = e - (e / np) * np;
    vidx[r][k] = (unsigned short)(slot_index(2 * k, r, m) | slot_index(2 * k + 1, r, m) << 8);
  }
  __syncthreads();
  // the first round's rotations (the slots hold the indices in order)
  if (tid < np) set_rotation(prm[0], tid, dg[2 * tid], dg[2 * tid + 1], A[2 * tid * LD + 2 * tid + 1], abs2);
  __syncthreads();

  // One round, reading buffer and rotation data PB, writing buffer and rotation data PB ^ 1.
  auto round = [&](auto pb_const, int r) {
    constexpr int PB = decltype(pb_const)::value;
    const RoundParams<NMAX> &P = prm[PB];
    // the other three entries of a block column, from the address of M[0][y] in buffer
    // PB: M[0][1-y] one column over, M[1][.] one row down
    constexpr int kColStep = PB ? LD : 1, kRowStep = PB ? 1 : LD;
    if (wave == 0) {
      // the next round's rotations (after the last round of a sweep: the first round
      // of the next one)
      if (lane < np) {
        const int base = PB ? rbase >> 16 : rbase & 0xffff;
        double bx, by;
        if (rflags & 8) {
          const double2 e1 = P.e[1];
          const double2 v = A[base];
          const bool rot = e1.x != 0.0 || e1.y != 0.0;
          bx = rot ? 0.0 : v.x;
          by = rot ? 0.0 : v.y;
        } else {
          const int ry = rflags & 1, d = ry ? -kColStep : kColStep;
          const double2 m0y = A[base], m0o = A[base + d];
          const double2 m1y = A[base + kRowStep], m1o = A[base + d + kRowStep];
          double2 o0, o1;
          block_column(m0y, m0o, m1y, m1o, P.cd[rx0].x, P.e[rx0 + 1], P.cd[rcq].x, P.e[rcq + 1], ry, o0, o1);
          const bool rx = rflags & 2;
          bx = rx ? o1.x : o0.x;
          by = rx ? o1.y : o0.y;
          by = (rflags & 4) ? -by : by;
        }
        const double a2 = P.cd[rs0].y, b2 = P.cd[rs1].y;
        set_rotation(prm[PB ^ 1], lane, a2, b2, make_double2(bx, by), abs2);
        dg[2 * lane] = a2;
        dg[2 * lane + 1] = b2;
      }
    } else if (wave <= BW) {
      // A <- J^H A J from buffer PB, written permuted into buffer PB ^ 1
#pragma unroll
      for (int u = 0; u < TPB; ++u) {
        // opaque to the compiler, so that the decoding below stays in the round (hoisted,
        // it would keep every task's addresses of both buffers in registers)
        int meta = bmeta[u], bb = bbase[u], ww0 = bw0[u], ww1 = bw1[u];
        asm volatile("" : "+v"(meta), "+v"(bb), "+v"(ww0), "+v"(ww1));
        const int kind = meta >> 24;
        if (kind == 0) continue;
        const int x0 = meta & 255, c0 = (meta >> 8) & 255;
        const int base = PB ? bb >> 16 : bb & 0xffff;
        const int wa = PB ? ww0 : ww1;
        if (kind == 1) {
          const double2 beta = A[base];
          const double2 e1 = P.e[c0];
          const bool rot = e1.x != 0.0 || e1.y != 0.0;
          A[wa & 0xffff] = rot ? make_double2(0.0, 0.0) : make_double2(beta.x, (meta >> 16) & 1 ? -beta.y : beta.y);
        } else {
          const int d = (c0 & 1) ? -kColStep : kColStep;
          const double2 m0y = A[base], m0o = A[base + d];
          const double2 m1y = A[base + kRowStep], m1o = A[base + d + kRowStep];
          double2 o0, o1;
          block_column(m0y, m0o, m1y, m1o, P.cd[x0].x, P.e[x0 + 1], P.cd[c0 & ~1].x, P.e[c0 | 1], c0 & 1, o0, o1);
          A[wa & 0xffff] = make_double2(o0.x, (meta >> 16) & 1 ? -o0.y : o0.y);
          A[wa >> 16] = make_double2(o1.x, (meta >> 17) & 1 ? -o1.y : o1.y);
        }
        __builtin_amdgcn_sched_barrier(0);
      }
    } else {
      // V <- V J in place: every operand is loaded first, then the items are rotated (a
      // pair that does not rotate has c = 1, e = 0 and is rotated all the same)
      double2 vp[VPT], vq[VPT], eq[VPT], ep[VPT];
      double cc[VPT];
      int ip[VPT], iq[VPT];
#pragma unroll
      for (int u = 0; u < VPT; ++u) {
        const int g = vwave + VW * u;
        const int k = g * GPW + vsub;
        const bool ok = g < NG && k < np && vrow < n;
        const int kk = ok ? k : 0, row = ok ? vrow : 0;
        const int pq = vidx[r][kk];
        ip[u] = ok ? row * LD + (pq & 255) : -1;
        iq[u] = row * LD + (pq >> 8);
        vp[u] = V[row * LD + (pq & 255)];
        vq[u] = V[iq[u]];
        cc[u] = P.cd[2 * kk].x;
        eq[u] = P.e[2 * kk + 1];  // J[p][q]
        ep[u] = P.e[2 * kk];      // J[q][p]
      }
#pragma unroll
      for (int u = 0; u < VPT; ++u) {
        if (ip[u] >= 0) {
          V[ip[u]] = zadd(zscale(vp[u], cc[u]), zmul(vq[u], ep[u]));
          V[iq[u]] = zadd(zmul(vp[u], eq[u]), zscale(vq[u], cc[u]));
        }
      }
    }
  };

  int sweeps = 0, pb = 0;  // pb: the buffer and the rotation data of the current round
  bool converged = false;
  for (;;) {
    // at the start of a sweep every index is on its own slot
    if (tid == 0) flag = 0;
    __syncthreads();
    for (int e = tid; e < n * n; e += kThreads) {
      const int i = e / n, j = e - (e / n) * n;
      if (i < j) {
        const double2 b = A[abuf_addr<LD>(pb, i, j)];
        const double ab2 = b.x * b.x + b.y * b.y;
        if (ab2 > kRelTol * kRelTol * fabs(dg[i] * dg[j]) && ab2 > abs2) flag = 1;
      }
    }
    __syncthreads();
    if (!flag) {
      converged = true;
      break;
    }
    if (sweeps >= max_sweeps) break;
    ++sweeps;
    for (int r = 0; r < m - 1; ++r) {
      if (pb)
        round(std::integral_constant<int, 1>{}, r);
      else
        round(std::integral_constant<int, 0>{}, r);
      __syncthreads();
      pb ^= 1;
    }
  }

  for (int i = tid; i < n; i += kThreads) A[i * LD + i] = make_double2(dg[i], 0.0);
  __syncthreads();
  store_sorted<NMAX>(pr, A, V, scale, rank_of, converged ? sweeps : -1);
}


// ---------------------------------------------------------------------------
// Step (c) by Householder reduction to real tridiagonal form and implicit QL,
// FP64, one workgroup of 256 threads per problem (n <= 64).
//  1. For k = 0 .. n-3 the reflector H_k = I - 2 u u^H (u unit, supported on
//     rows k+1 ..) maps column k below the diagonal to alpha_k e_1, |alpha_k| =
//     its norm, with the phase chosen opposite to its first entry (no
//     cancellation).  The trailing block B becomes B - u w^H - w u^H,
//     w = 2 (p - (u^H p) u), p = B u.  u_k is kept in column k of A.
//  2. V = H_0 H_1 ... H_{n-3} (applied right to left to the identity), then the
//     diagonal unitary D with delta_{k+1} = delta_k alpha_k / |alpha_k| makes the
//     off-diagonals real and non-negative: A = (V D) T (V D)^H.
//  3. Implicit QL with Wilkinson-type shifts on the real tridiagonal T (wave 0:
//     every lane runs the same scalar recurrence, lane r applies each plane
//     rotation to row r of V D).
// info = the number of QL iterations, or -1 if one eigenvalue needed more than
// max_iter of them.
template <int NMAX>
__global__ __launch_bounds__(256) void eigh_tridiag(EighBatch batch, int max_iter) {
  constexpr int kThreads = 256, LD = NMAX + 1, G = kThreads / 64;
  const EighProblem &pr = batch.prob[blockIdx.x];
  const int n = pr.n;
  extern __shared__ double2 smem[];
  double2 *const A = smem;              // [n][LD]
  double2 *const V = smem + NMAX * LD;  // [n][LD]
  __shared__ double2 part[G][64];
  __shared__ double2 wv[64];
  __shared__ double2 alpha[NMAX];
  __shared__ double dg[NMAX], od[NMAX];
  __shared__ double red[kThreads];
  __shared__ int rank_of[NMAX];
  const int tid = threadIdx.x, lane = tid & 63, grp = tid >> 6;

  const double scale = load_scaled<NMAX, kThreads>(pr, A, V, red);

  // 1. Householder reduction
  for (int k = 0; k + 2 < n; ++k) {
    const int m = n - k - 1;
    if (tid < 64) {
      const double2 x = lane < m ? A[(k + 1 + lane) * LD + k] : make_double2(0.0, 0.0);
      double s2 = x.x * x.x + x.y * x.y;
#pragma unroll
      for (int o = 32; o > 0; o >>= 1) s2 += __shfl_xor(s2, o);
      const double x0r = __shfl(x.x, 0), x0i = __shfl(x.y, 0);
      const double ax0 = sqrt(x0r * x0r + x0i * x0i);
      const double an = sqrt(s2);
      double2 u = make_double2(0.0, 0.0), al = make_double2(0.0, 0.0);
      if (an > 0.0) {
        const double phr = ax0 > 0.0 ? x0r / ax0 : 1.0, phi = ax0 > 0.0 ? x0i / ax0 : 0.0;
        al = make_double2(-phr * an, -phi * an);
        const double inv = 1.0 / sqrt(2.0 * an * (an + ax0));
        const double2 v = lane == 0 ? make_double2(x.x - al.x, x.y - al.y) : x;
        u = make_double2(v.x * inv, v.y * inv);
      }
      if (lane < m) A[(k + 1 + lane) * LD + k] = u;
      if (lane == 0) alpha[k] = al;
    }
    __syncthreads();
    // p = B u: group g sums the columns j = g, g + G, ... of row `lane`
    if (lane < m) {
      double2 acc = make_double2(0.0, 0.0);
      const double2 *row = A + (k + 1 + lane) * LD + (k + 1);
      for (int j = grp; j < m; j += G) acc = zadd(acc, zmul(row[j], A[(k + 1 + j) * LD + k]));
      part[grp][lane] = acc;
    }
    __syncthreads();
    if (tid < 64) {
      double2 p = make_double2(0.0, 0.0);
      const double2 u = lane < m ? A[(k + 1 + lane) * LD + k] : make_double2(0.0, 0.0);
      if (lane < m) {
#pragma unroll
        for (int g = 0; g < G; ++g) p = zadd(p, part[g][lane]);
      }
      double kk = u.x * p.x + u.y * p.y;  // Re(conj(u) p)
#pragma unroll
      for (int o = 32; o > 0; o >>= 1) kk += __shfl_xor(kk, o);
      if (lane < m) wv[lane] = make_double2(2.0 * (p.x - kk * u.x), 2.0 * (p.y - kk * u.y));
    }
    __syncthreads();
    // B <- B - u w^H - w u^H
    for (int e = tid; e < m * m; e += kThreads) {
      const int i = e / m, j = e - (e / m) * m;
      const double2 ui = A[(k + 1 + i) * LD + k], uj = A[(k + 1 + j) * LD + k];
      const double2 wi = wv[i], wj = wv[j];
      double2 &b = A[(k + 1 + i) * LD + (k + 1 + j)];
      b = zsub(b, zadd(zmul(ui, zconj(wj)), zmul(wi, zconj(uj))));
    }
    __syncthreads();
  }

  // 2. V = H_0 ... H_{n-3} from the right end, then the phases
  for (int k = n - 3; k >= 0; --k) {
    const int m = n - k - 1;
    // s_c = sum_i conj(u_i) V[k+1+i][c] for the columns c = k+1 .. n-1
    if (lane < m) {
      double2 acc = make_double2(0.0, 0.0);
      for (int i = grp; i < m; i += G) acc = zadd(acc, zmul(zconj(A[(k + 1 + i) * LD + k]), V[(k + 1 + i) * LD + (k + 1 + lane)]));
      part[grp][lane] = acc;
    }
    __syncthreads();
    if (tid < 64 && lane < m) {
      double2 sc = make_double2(0.0, 0.0);
#pragma unroll
      for (int g = 0; g < G; ++g) sc = zadd(sc, part[g][lane]);
      wv[lane] = sc;
    }
    __syncthreads();
    for (int e = tid; e < m * m; e += kThreads) {
      const int i = e / m, c = e - (e / m) * m;
      const double2 ui = A[(k + 1 + i) * LD + k];
      double2 &v = V[(k + 1 + i) * LD + (k + 1 + c)];
      const double2 t = zmul(ui, wv[c]);
      v = make_double2(v.x - 2.0 * t.x, v.y - 2.0 * t.y);
    }
    __syncthreads();
  }
  if (tid == 0) {
    // real tridiagonal: diagonal, off-diagonal |alpha_k|; the phases delta_k go to wv
    for (int i = 0; i < n; ++i) dg[i] = A[i * LD + i].x;
    double2 dl = make_double2(1.0, 0.0);
    wv[0] = dl;
    for (int k = 0; k + 1 < n; ++k) {
      const double2 a = k + 2 < n ? alpha[k] : A[(k + 1) * LD + k];
      const double aa = sqrt(a.x * a.x + a.y * a.y);
      od[k] = aa;
      if (aa > 0.0) dl = zmul(dl, make_double2(a.x / aa, a.y / aa));
      wv[k + 1] = dl;
    }
    od[n - 1] = 0.0;
  }
  __syncthreads();
  for (int e = tid; e < n * n; e += kThreads) {
    const int i = e / n, j = e - (e / n) * n;
    V[i * LD + j] = zmul(V[i * LD + j], wv[j]);
  }
  __syncthreads();

  // 3. implicit QL on (dg, od), wave 0.  Lane j keeps d_j and e_j in registers; the
  // scalar recurrence (identical on every lane) reads them with readlane and writes
  // them back with a lane select.  A sweep's plane rotations are kept in LDS and
  // then applied to the rows of V D (lane r, row r) with the running column held in
  // registers.
  if (tid < 64) {
    const double eps = 2.220446049250313e-16;
    double dL = lane < n ? dg[lane] : 0.0, eL = lane < n ? od[lane] : 0.0;
    auto rd = [](double x, int j) {  // x of lane j (j wave-uniform)
      return __hiloint2double(__builtin_amdgcn_readlane(__double2hiint(x), j),
                              __builtin_amdgcn_readlane(__double2loint(x), j));
    };
    int total = 0;
    bool ok = true;
    for (int l = 0; l < n && ok; ++l) {
      int iter = 0;
      for (;;) {
        int m = l;
        while (m + 1 < n && fabs(rd(eL, m)) > eps * (fabs(rd(dL, m)) + fabs(rd(dL, m + 1)))) ++m;
        if (m == l) break;
        if (iter == max_iter) {
          ok = false;
          break;
        }
        ++iter;
        ++total;
        const double el = rd(eL, l), dl = rd(dL, l);
        double g = (rd(dL, l + 1) - dl) / (2.0 * el);
        double r = sqrt(g * g + 1.0);
        g = rd(dL, m) - dl + el / (g + (g >= 0.0 ? r : -r));
        double sn = 1.0, cs = 1.0, p = 0.0;
        int last = l;  // lowest rotated index + 1 .. m: columns last .. m change
        bool split = false;
        for (int i = m - 1; i >= l; --i) {
          const double ei = rd(eL, i);
          const double f = sn * ei, b = cs * ei;
          const double r2 = f * f + g * g;
          if (r2 == 0.0) {  // the matrix split at i: restart on the reduced problem
            const double di1 = rd(dL, i + 1) - p;
            if (lane == i + 1) { dL = di1; eL = 0.0; }
            if (lane == m) eL = 0.0;
            last = i + 1;
            split = true;
            break;
          }
          const double ir = rsq64(r2);
          r = r2 * ir;
          if (lane == i + 1) eL = r;
          sn = f * ir;
          cs = g * ir;
          const double di = rd(dL, i);
          g = rd(dL, i + 1) - p;
          r = (di - g) * sn + 2.0 * cs * b;
          p = sn * r;
          if (lane == i + 1) dL = g + p;
          g = cs * r - b;
          if (lane == 0) {
            wv[i] = make_double2(cs, sn);
          }
          last = i;
        }
        // the rotations i = m-1 .. last, in that order, on the rows of V
        if (lane < n && last < m) {
          double2 hi = V[lane * LD + m];
          for (int i = m - 1; i >= last; --i) {
            const double2 q = wv[i];  // (c, s)
            const double2 lo = V[lane * LD + i];
            V[lane * LD + i + 1] = make_double2(q.y * lo.x + q.x * hi.x, q.y * lo.y + q.x * hi.y);
            hi = make_double2(q.x * lo.x - q.y * hi.x, q.x * lo.y - q.y * hi.y);
          }
          V[lane * LD + last] = hi;
        }
        if (split) continue;
        if (lane == l) { dL -= p; eL = g; }
        if (lane == m) eL = 0.0;
      }
    }
    if (lane < n) dg[lane] = dL;
    if (lane == 0) red[0] = ok ? (double)total : -1.0;
  }
  __syncthreads();
  const int info_value = (int)red[0];
  for (int i = tid; i < n; i += kThreads) A[i * LD + i] = make_double2(dg[i], 0.0);
  __syncthreads();
  store_sorted<NMAX>(pr, A, V, scale, rank_of, info_value);
}

template <int NMAX>
constexpr size_t eigh_static_lds() {
  return 2 * sizeof(RoundParams<NMAX>) + sizeof(int) + threads_for<NMAX>() * sizeof(double) + NMAX * sizeof(int) +
         NMAX * sizeof(double) + (NMAX - 1) * (NMAX / 2) * sizeof(unsigned short) + 512;
}

template <int NMAX>
hipError_t launch_batch(const EighBatch &b, int count, int max_sweeps, hipStream_t s) {
  static bool attr_set[64] = {};
  int dev = 0;
  hipError_t e = hipGetDevice(&dev);
  if (e != hipSuccess) return e;
  // The whole CU's LDS is requested so that no other workgroup (all the other
  // kernels of the path use LDS) shares the CU with this latency-bound kernel.
  const size_t shmem = kCuLdsBytes - eigh_static_lds<NMAX>();
  if (dev < 0 || dev >= 64 || !attr_set[dev]) {
    e = hipFuncSetAttribute((const void *)eigh_jacobi<NMAX>, hipFuncAttributeMaxDynamicSharedMemorySize,
                            (int)shmem);
    if (e != hipSuccess) return e;
    if (dev >= 0 && dev < 64) attr_set[dev] = true;
  }
  ProfScope ps("eigh_jacobi", s);
  hipLaunchKernelGGL((eigh_jacobi<NMAX>), dim3(count), dim3(threads_for<NMAX>()), shmem, s, b, max_sweeps);
  return hipGetLastError();
}

template <int NMAX>
hipError_t launch_tridiag(const EighBatch &b, int count, int max_iter, hipStream_t s) {
  static bool attr_set[64] = {};
  int dev = 0;
  hipError_t e = hipGetDevice(&dev);
  if (e != hipSuccess) return e;
  const size_t shmem = 2 * (size_t)NMAX * (NMAX + 1) * sizeof(double2);  // A and V
  if (dev < 0 || dev >= 64 || !attr_set[dev]) {
    e = hipFuncSetAttribute((const void *)eigh_tridiag<NMAX>, hipFuncAttributeMaxDynamicSharedMemorySize,
                            (int)shmem);
    if (e != hipSuccess) return e;
    if (dev >= 0 && dev < 64) attr_set[dev] = true;
  }
  ProfScope ps("eigh_tridiag", s);
  hipLaunchKernelGGL((eigh_tridiag<NMAX>), dim3(count), dim3(256), shmem, s, b, max_iter);
  return hipGetLastError();
}

}  // namespace

hipError_t launch_eigh_batch(const EighProblem *probs, int count, int max_iter, hipStream_t s) {
  // problems go to the kernel of their method and size class (n <= 32, n <= 64),
  // at most kMaxEighBatch per launch
  for (int method : {HH_EIGH_JACOBI, HH_EIGH_TRIDIAG}) {
    for (int big = 0; big < 2; ++big) {
      EighBatch b{};
      int m = 0;
      auto flush = [&]() -> hipError_t {
        hipError_t e = hipSuccess;
        if (m == 0) return e;
        if (method == HH_EIGH_JACOBI)
          e = big ? launch_batch<64>(b, m, max_iter, s) : launch_batch<32>(b, m, max_iter, s);
        else
          e = big ? launch_tridiag<64>(b, m, max_iter, s) : launch_tridiag<32>(b, m, max_iter, s);
        m = 0;
        return e;
      };
      for (int i = 0; i < count; ++i) {
        if ((probs[i].n > 32) != (big == 1) || probs[i].method != method) continue;
        b.prob[m++] = probs[i];
        if (m == kMaxEighBatch) {
          const hipError_t e = flush();
          if (e != hipSuccess) return e;
        }
      }
      const hipError_t e = flush();
      if (e != hipSuccess) return e;
    }
  }
  return hipSuccess;
}

hipError_t launch_eigh(int nt, const double *cov, double *evals, double *evecs, int *info, int max_sweeps,
                       hipStream_t s) {
  EighProblem p{nt, cov, evals, evecs, info};
  p.method = HH_EIGH_JACOBI;
  return launch_eigh_batch(&p, 1, max_sweeps, s);
}

}  // namespace hh
