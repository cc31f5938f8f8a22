// Step (c), Eq. (5): C = V Lambda V^{t*} by parallel cyclic Jacobi in FP64, one workgroup.
//
// A sweep is m-1 rounds (m = n rounded up to even) of m/2 disjoint 2x2 Hermitian
// rotations (round-robin pairing: every index pair once per sweep).  For a pair
// (p, q) with a = A[p][p], b = A[q][q], beta = A[p][q], g = b - a:
//   D = sqrt(g^2 + 4 |beta|^2),  den = sqrt(2 D (D + |g|)),
//   c = (D + |g|) / den,  J[p][q] = sgn(g) 2 beta / den,  J[q][p] = -conj(J[p][q]),
//   J[p][p] = J[q][q] = c,   A <- J^H A J,   V <- V J,
// which zeroes A[p][q] and moves t|beta| = sgn(g) 2 |beta|^2 / (D + |g|) from A[p][p]
// to A[q][q] (the textbook t = sgn(theta)/(|theta| + sqrt(1 + theta^2)),
// theta = g / (2|beta|), rewritten to need two square roots and one division).
//
// Work split per round: (1) every thread rotates the 2x2 blocks {p1,q1} x {p2,q2}
// of A it owns, in place (the four outputs share the four inputs; only the upper
// triangle of A is kept, so each entry is read and written once); barrier;
// (2) wave 0 computes the next round's rotations from three entries each, with
// hardware reciprocal / reciprocal-square-root seeds refined by Newton steps,
// while the other waves rotate V's (row, pair) entries in place, one row per lane
// and one pair per group of lanes (the group's rotation data is one LDS
// broadcast); barrier.  C is scaled by an exact power of two so that its Frobenius
// norm is O(1).
// A rotation is skipped when |beta| <= 1e-15 sqrt(|a b|) or |beta| <= 1e-18 ||C||_F;
// the iteration stops when every off-diagonal entry passes that test.  The result
// is sorted by decreasing eigenvalue and each eigenvector's phase is fixed.
#include "hh_internal.h"

namespace hh {
namespace {

constexpr double kRelTol = 1e-15;
constexpr double kAbsTol = 1e-18;
// threads per problem: 576 for n <= 32 (rounds are latency-bound; wave 0 computes
// the rotations while eight waves rotate V, one (row, pair) item each), 1024 for
// n <= 64 (a round has four times the 2x2 blocks and V items, so it is throughput-bound)
template <int NMAX>
constexpr int threads_for() { return NMAX <= 32 ? 576 : 1024; }
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

// Per-round rotation data, indexed by matrix index i: cd[i] = (c_i, new diagonal
// entry i), e[i] = J[partner][i].  A pair rotates iff its e is nonzero (a rotating
// pair has |beta| > 1e-18 ||C||_F after scaling, so e cannot underflow to zero);
// a pair that does not rotate has c = 1, e = 0 and its diagonal entries as they are.
template <int NMAX>
struct RoundParams {
  double2 cd[NMAX];
  double2 e[NMAX];
};

// Round-robin pairing: pair k of round r among m players (p < q; q may be the dummy).
__device__ __forceinline__ void pair_of(int r, int k, int m, int &p, int &q) {
  if (k == 0) {
    p = r;
    q = m - 1;
  } else {  // (r + k) mod (m - 1) and (r - k) mod (m - 1), with 0 <= r < m - 1, 0 < k < m / 2
    p = r + k >= m - 1 ? r + k - (m - 1) : r + k;
    q = r - k < 0 ? r - k + (m - 1) : r - k;
  }
  if (p > q) {
    const int x = p;
    p = q;
    q = x;
  }
}

template <int NMAX>
__device__ __forceinline__ void set_rotation(RoundParams<NMAX> &P, int p, int q, int n, double a, double b,
                                             double2 beta, double abs2) {
  if (q >= n) {  // paired with the dummy index: no rotation
    P.cd[p] = make_double2(1.0, a);
    P.e[p] = make_double2(0.0, 0.0);
    return;
  }
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
  P.cd[p] = make_double2(c, rot ? a - tab : a);
  P.cd[q] = make_double2(c, rot ? b + tab : b);
  P.e[q] = eq;
  P.e[p] = rot ? make_double2(-eq.x, eq.y) : make_double2(0.0, 0.0);  // J[q][p] = -conj(J[p][q])
}

// Entry (i, j) of the Hermitian A, of which only the upper triangle (i <= j) is
// kept up to date.
__device__ __forceinline__ double2 herm(const double2 *A, int LD, int i, int j) {
  const bool up = i <= j;
  const double2 v = A[(up ? i : j) * LD + (up ? j : i)];
  return make_double2(v.x, up ? v.y : -v.y);
}
// Writes entry (i, j) at its upper-triangle position.
__device__ __forceinline__ void herm_store(double2 *A, int LD, int i, int j, double2 v) {
  const bool up = i <= j;
  A[(up ? i : j) * LD + (up ? j : i)] = make_double2(v.x, up ? v.y : -v.y);
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
  // one workgroup per problem of the batch
  const EighProblem &pr = batch.prob[blockIdx.x];
  const int n = pr.n;
  constexpr int LD = NMAX + 1;
  constexpr int NPMAX = NMAX / 2;
  constexpr int NBLK = NPMAX * (NPMAX + 1) / 2;
  constexpr int BPT = (NBLK + kThreads - 1) / kThreads;          // A blocks per thread
  extern __shared__ double2 smem[];
  double2 *const A = smem;              // [n][LD]
  double2 *const V = smem + NMAX * LD;  // [n][LD]
  __shared__ RoundParams<NMAX> prm[2];
  __shared__ int flag;
  __shared__ double red[kThreads];
  __shared__ int rank_of[NMAX];
  const int tid = threadIdx.x;
  const int m = n + (n & 1);
  const int np = m / 2;
  const int nblk = np * (np + 1) / 2;

  // blocks (P <= Q) owned by this thread, unranked once
  int bP[BPT], bQ[BPT];
#pragma unroll
  for (int u = 0; u < BPT; ++u) {
    int b = tid + kThreads * u, P = 0;
    bP[u] = -1;
    bQ[u] = -1;
    if (b < nblk) {
      while (b >= np - P) {
        b -= np - P;
        ++P;
      }
      bP[u] = P;
      bQ[u] = P + b;
    }
  }

  // V items: waves 1.. rotate V with one row per lane, the wave's lanes in groups of
  // NMAX rows that each take one pair, so the rotation data a group reads is one
  // LDS broadcast.  Item g of a wave is the pairs GPW g .. GPW g + GPW - 1.
  constexpr int GPW = 64 / NMAX;                  // pairs per wave and item
  constexpr int VW = kThreads / 64 - 1;           // waves rotating V
  constexpr int NG = NPMAX / GPW;                 // items
  constexpr int VPT = (NG + VW - 1) / VW;         // items per wave
  const int vrow = (tid & 63) % NMAX, vsub = (tid & 63) / NMAX, vwave = (tid >> 6) - 1;

  const double scale = load_scaled<NMAX, kThreads>(pr, A, V, red);
  const double fro = red[0] / scale;  // Frobenius norm of C (exactly, scale is a power of two)
  const double abs2 = (kAbsTol * fro * scale) * (kAbsTol * fro * scale);
  __syncthreads();

  int sweeps = 0;
  bool converged = false;
  for (;;) {
    if (tid == 0) flag = 0;
    __syncthreads();
    for (int e = tid; e < n * n; e += kThreads) {
      const int i = e / n, j = e - (e / n) * n;
      if (i < j) {
        const double2 b = A[i * LD + j];
        const double ab2 = b.x * b.x + b.y * b.y;
        if (ab2 > kRelTol * kRelTol * fabs(A[i * LD + i].x * A[j * LD + j].x) && ab2 > abs2) flag = 1;
      }
    }
    __syncthreads();
    if (!flag) {
      converged = true;
      break;
    }
    if (sweeps >= max_sweeps) break;
    ++sweeps;

    if (tid < np) {
      int p, q;
      pair_of(0, tid, m, p, q);
      const int qc = q < n ? q : p;
      set_rotation(prm[0], p, q, n, A[p * LD + p].x, A[qc * LD + qc].x, A[p * LD + qc], abs2);
    }
    __syncthreads();

    int pb = 0;
    for (int r = 0; r < m - 1; ++r) {
      const RoundParams<NMAX> &P = prm[pb];
      // (1) A <- J^H A J on the blocks this thread owns (in place: an entry of the upper
      // triangle belongs to one block)
#pragma unroll
      for (int u = 0; u < BPT; ++u) {
        if (bP[u] < 0) continue;
        // the pairing is fixed arithmetic: recomputed in registers (no dependent LDS read)
        int p1, q1, p2, q2;
        pair_of(r, bP[u], m, p1, q1);
        pair_of(r, bQ[u], m, p2, q2);
        // One instruction stream for the pair's own block (P == Q) and the others:
        // every operand is loaded first; on the own block of a rotating pair the
        // rotated values are replaced by the exact ones (zero off-diagonal, moved
        // diagonal).  A pair that does not rotate has c = 1, e = 0, for which the
        // products below return its entries unchanged.
        const bool own = bP[u] == bQ[u];
        const bool vq1 = q1 < n, vq2 = q2 < n;
        // value selects (clamped indices), never a select between LDS and a local
        const int q1c = vq1 ? q1 : p1, q2c = vq2 ? q2 : p2;
        const double m1 = vq1 ? 1.0 : 0.0, m2 = vq2 ? 1.0 : 0.0;
        const double2 a = herm(A, LD, p1, p2);
        const double2 b = zscale(herm(A, LD, p1, q2c), m2);
        const double2 d = zscale(herm(A, LD, q1c, p2), m1);
        const double2 f = zscale(herm(A, LD, q1c, q2c), m1 * m2);
        const double2 cd1 = P.cd[p1];
        const double c1 = cd1.x, dp = cd1.y, dq = P.cd[q1c].y, c2 = P.cd[p2].x;
        const double2 e1 = zscale(P.e[q1c], m1);  // J[p1][q1]
        const double2 e2 = zscale(P.e[q2c], m2);  // J[p2][q2]
        const bool rot = e1.x != 0.0 || e1.y != 0.0;
        // T = M J2 (columns p2, q2), then J1^H T (rows p1, q1)
        const double2 me2c = make_double2(-e2.x, e2.y);  // J[q2][p2]
        const double2 t00 = zadd(zscale(a, c2), zmul(b, me2c)), t01 = zadd(zmul(a, e2), zscale(b, c2));
        const double2 t10 = zadd(zscale(d, c2), zmul(f, me2c)), t11 = zadd(zmul(d, e2), zscale(f, c2));
        double2 o00 = zsub(zscale(t00, c1), zmul(e1, t10));
        double2 o01 = zsub(zscale(t01, c1), zmul(e1, t11));
        const double2 e1c = zconj(e1);
        const double2 o10 = zadd(zmul(e1c, t00), zscale(t10, c1));
        double2 o11 = zadd(zmul(e1c, t01), zscale(t11, c1));
        if (own && rot) {
          o00 = make_double2(dp, 0.0);
          o11 = make_double2(dq, 0.0);
          o01 = make_double2(0.0, 0.0);
        }
        herm_store(A, LD, p1, p2, o00);
        if (vq2) herm_store(A, LD, p1, q2, o01);
        if (vq1 && !own) herm_store(A, LD, q1, p2, o10);  // on the own block: o01's entry
        if (vq1 && vq2) herm_store(A, LD, q1, q2, o11);
      }
      __syncthreads();
      if (tid < 64) {
        // (2a) wave 0: the next round's rotations from the updated A
        if (r + 1 < m - 1 && tid < np) {
          int p, q;
          pair_of(r + 1, tid, m, p, q);
          const int qc = q < n ? q : p;
          set_rotation(prm[pb ^ 1], p, q, n, A[p * LD + p].x, A[qc * LD + qc].x, A[p * LD + qc], abs2);
        }
      } else {
        // (2b) waves 1..: V <- V J, one (row, pair) entry pair per lane and item; every
        // operand is loaded first, then the items are rotated (a pair that does not
        // rotate has c = 1, e = 0 and is rotated all the same)
        double2 vp[VPT], vq[VPT], eq[VPT], ep[VPT];
        double cc[VPT];
        int ip[VPT], iq[VPT];
#pragma unroll
        for (int u = 0; u < VPT; ++u) {
          const int k = (vwave + VW * u) * GPW + vsub;
          const bool ok = vwave + VW * u < NG && k < np && vrow < n;
          int p = 0, q = 0;
          if (ok) pair_of(r, k, m, p, q);
          const int row = ok ? vrow : 0;
          const int qc = q < n ? q : p;
          ip[u] = row * LD + p;
          iq[u] = ok && q < n ? row * LD + q : -1;
          vp[u] = V[row * LD + p];
          vq[u] = V[row * LD + qc];
          cc[u] = P.cd[p].x;
          eq[u] = P.e[qc];  // J[p][q]
          ep[u] = P.e[p];   // J[q][p]
        }
#pragma unroll
        for (int u = 0; u < VPT; ++u) {
          if (iq[u] >= 0) {
            V[ip[u]] = zadd(zscale(vp[u], cc[u]), zmul(vq[u], ep[u]));
            V[iq[u]] = zadd(zmul(vp[u], eq[u]), zscale(vq[u], cc[u]));
          }
        }
      }
      __syncthreads();
      pb ^= 1;
    }
  }

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
  return 2 * sizeof(RoundParams<NMAX>) + sizeof(int) + threads_for<NMAX>() * sizeof(double) + NMAX * sizeof(int) + 512;
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
