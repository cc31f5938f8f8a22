// Step (c), Eq. (5): C = V Lambda V^{t*} by parallel cyclic Jacobi in FP64, one workgroup.
//
// Each round applies n/2 disjoint 2x2 Hermitian rotations (round-robin pairing,
// every pair once per sweep).  For the pair (p, q) with beta = A[p][q] = |beta| e^{i phi}:
//   theta = (A[q][q] - A[p][p]) / (2 |beta|),  t = sgn(theta) / (|theta| + sqrt(1 + theta^2)),
//   c = 1 / sqrt(1 + t^2),  s = t c,
//   J = [[c, s e^{i phi}], [-s e^{-i phi}, c]],  A <- J^H A J,  V <- V J,
// which zeroes A[p][q] and moves t|beta| between the two diagonal entries.
// Rotations are skipped when |beta| <= 1e-15 sqrt(|A[p][p] A[q][q]|); the sweep
// loop stops when every off-diagonal entry passes that test.  The result is
// sorted by decreasing eigenvalue and each eigenvector's phase is fixed.
#include "hh_internal.h"

namespace hh {
namespace {

constexpr double kRelTol = 1e-15;
constexpr double kTiny = 1e-300;
constexpr int kMaxN = 64;
constexpr int kThreads = 256;
constexpr int kPer = kMaxN * kMaxN / kThreads;  // elements per thread per matrix

__device__ __forceinline__ double2 zmul(double2 a, double2 b) {
  return make_double2(a.x * b.x - a.y * b.y, a.x * b.y + a.y * b.x);
}
__device__ __forceinline__ double2 zconj(double2 a) { return make_double2(a.x, -a.y); }
__device__ __forceinline__ double2 zscale(double2 a, double s) { return make_double2(a.x * s, a.y * s); }
__device__ __forceinline__ double2 zadd(double2 a, double2 b) { return make_double2(a.x + b.x, a.y + b.y); }

__global__ __launch_bounds__(kThreads) void eigh_jacobi(int n, const double2 *__restrict__ C,
                                                        double *__restrict__ evals, double2 *__restrict__ evecs,
                                                        int *__restrict__ info, int max_sweeps) {
  extern __shared__ double2 smem[];
  const int ld = n + 1;
  double2 *A = smem;            // [n][ld]
  double2 *V = smem + n * ld;   // [n][ld]
  __shared__ int partner[kMaxN];
  __shared__ int rotated[kMaxN];
  __shared__ double cc[kMaxN];
  __shared__ double2 ee[kMaxN];
  __shared__ double dnew[kMaxN];
  __shared__ int rank_of[kMaxN];
  __shared__ int not_done;
  const int tid = threadIdx.x;
  const int m = n + (n & 1);  // even number of players (one dummy if n is odd)

  // Hermitian input: the lower triangle and the real diagonal are read.
  for (int e = tid; e < n * n; e += kThreads) {
    const int i = e / n, j = e % n;
    double2 a;
    if (i > j) a = C[i * n + j];
    else if (i < j) a = zconj(C[j * n + i]);
    else a = make_double2(C[i * n + i].x, 0.0);
    A[i * ld + j] = a;
    V[i * ld + j] = make_double2(i == j ? 1.0 : 0.0, 0.0);
  }
  __syncthreads();

  int sweeps = 0;
  bool converged = false;
  for (;;) {
    // convergence test over all off-diagonal pairs
    if (tid == 0) not_done = 0;
    __syncthreads();
    for (int e = tid; e < n * n; e += kThreads) {
      const int i = e / n, j = e % n;
      if (i < j) {
        const double2 b = A[i * ld + j];
        const double ab = sqrt(b.x * b.x + b.y * b.y);
        const double th = kRelTol * sqrt(fabs(A[i * ld + i].x * A[j * ld + j].x));
        if (ab > th && ab > kTiny) not_done = 1;
      }
    }
    __syncthreads();
    if (!not_done) { converged = true; break; }
    if (sweeps >= max_sweeps) break;
    ++sweeps;

    for (int r = 0; r < m - 1; ++r) {
      // (1) rotation parameters, one pair per thread
      if (tid < m / 2) {
        int p, q;
        if (tid == 0) { p = r; q = m - 1; }
        else { p = (r + tid) % (m - 1); q = (r - tid + m - 1) % (m - 1); }
        if (p > q) { const int x = p; p = q; q = x; }
        if (q >= n) {  // paired with the dummy player: no rotation
          partner[p] = p; cc[p] = 1.0; ee[p] = make_double2(0.0, 0.0); rotated[p] = 0;
        } else {
          const double a = A[p * ld + p].x, b = A[q * ld + q].x;
          const double2 beta = A[p * ld + q];
          const double ab = sqrt(beta.x * beta.x + beta.y * beta.y);
          partner[p] = q; partner[q] = p;
          if (ab > kRelTol * sqrt(fabs(a * b)) && ab > kTiny) {
            const double theta = (b - a) / (2.0 * ab);
            double t;
            if (fabs(theta) > 1e150) t = 0.5 / theta;
            else t = (theta >= 0.0 ? 1.0 : -1.0) / (fabs(theta) + sqrt(1.0 + theta * theta));
            const double c = 1.0 / sqrt(1.0 + t * t), s = t * c;
            const double2 ph = make_double2(beta.x / ab, beta.y / ab);  // e^{i phi}
            cc[p] = c; cc[q] = c;
            ee[p] = zscale(zconj(ph), -s);  // J[q][p]
            ee[q] = zscale(ph, s);          // J[p][q]
            dnew[p] = a - t * ab; dnew[q] = b + t * ab;
            rotated[p] = 1; rotated[q] = 1;
          } else {
            cc[p] = 1.0; cc[q] = 1.0;
            ee[p] = make_double2(0.0, 0.0); ee[q] = make_double2(0.0, 0.0);
            rotated[p] = 0; rotated[q] = 0;
          }
        }
      }
      __syncthreads();
      // (2) new entries into registers: A' = J^H A J (upper triangle), V' = V J
      double2 na[kPer], nv[kPer];
#pragma unroll
      for (int u = 0; u < kPer; ++u) {
        const int e = tid + kThreads * u;
        if (e < n * n) {
          const int i = e / n, j = e % n;
          const int ip = partner[i], jp = partner[j];
          const double ci = cc[i], cj = cc[j];
          const double2 ei = ee[i], ej = ee[j];
          if (i <= j) {
            double2 x;
            if (i == j) {
              x = rotated[i] ? make_double2(dnew[i], 0.0) : make_double2(A[i * ld + i].x, 0.0);
            } else if (j == ip && rotated[i]) {
              x = make_double2(0.0, 0.0);
            } else {
              x = zscale(A[i * ld + j], ci * cj);
              x = zadd(x, zmul(zscale(ej, ci), A[i * ld + jp]));
              const double2 eic = zconj(ei);
              x = zadd(x, zmul(zscale(eic, cj), A[ip * ld + j]));
              x = zadd(x, zmul(zmul(eic, ej), A[ip * ld + jp]));
            }
            na[u] = x;
          }
          nv[u] = zadd(zscale(V[i * ld + j], cj), zmul(V[i * ld + jp], ej));
        }
      }
      __syncthreads();
      // (3) write back, mirroring the upper triangle
#pragma unroll
      for (int u = 0; u < kPer; ++u) {
        const int e = tid + kThreads * u;
        if (e < n * n) {
          const int i = e / n, j = e % n;
          if (i <= j) {
            A[i * ld + j] = na[u];
            if (i < j) A[j * ld + i] = zconj(na[u]);
          }
          V[i * ld + j] = nv[u];
        }
      }
      __syncthreads();
    }
  }

  // sort by decreasing eigenvalue (ties: lower index first)
  if (tid < n) {
    const double di = A[tid * ld + tid].x;
    int rk = 0;
    for (int j = 0; j < n; ++j) {
      const double dj = A[j * ld + j].x;
      rk += (dj > di) || (dj == di && j < tid);
    }
    rank_of[tid] = rk;
    evals[rk] = di;
  }
  __syncthreads();
  // phase fix: the lowest row whose modulus is within 1e-12 of the largest becomes real > 0
  if (tid < n) {
    const int k = tid, col = rank_of[k];
    double mx = 0.0;
    for (int j = 0; j < n; ++j) {
      const double2 v = V[j * ld + k];
      mx = fmax(mx, sqrt(v.x * v.x + v.y * v.y));
    }
    int js = 0;
    for (int j = n - 1; j >= 0; --j) {
      const double2 v = V[j * ld + k];
      if (sqrt(v.x * v.x + v.y * v.y) >= mx * (1.0 - 1e-12)) js = j;
    }
    const double2 vs = V[js * ld + k];
    const double ms = sqrt(vs.x * vs.x + vs.y * vs.y);
    const double2 ph = ms > 0.0 ? make_double2(vs.x / ms, -vs.y / ms) : make_double2(1.0, 0.0);
    for (int j = 0; j < n; ++j) {
      const double2 v = (j == js) ? make_double2(ms, 0.0) : zmul(V[j * ld + k], ph);
      evecs[j * n + col] = v;
    }
  }
  if (tid == 0) *info = converged ? sweeps : -1;
}

}  // namespace

hipError_t launch_eigh(int nt, const double *cov, double *evals, double *evecs, int *info, int max_sweeps,
                       hipStream_t s) {
  const size_t shmem = 2 * (size_t)nt * (nt + 1) * sizeof(double2);
  static bool attr_set[64] = {};
  int dev = 0;
  hipError_t e = hipGetDevice(&dev);
  if (e != hipSuccess) return e;
  if (dev < 0 || dev >= 64 || !attr_set[dev]) {
    e = hipFuncSetAttribute((const void *)eigh_jacobi, hipFuncAttributeMaxDynamicSharedMemorySize,
                            2 * kMaxN * (kMaxN + 1) * (int)sizeof(double2));
    if (e != hipSuccess) return e;
    if (dev >= 0 && dev < 64) attr_set[dev] = true;
  }
  ProfScope ps("eigh_jacobi", s);
  hipLaunchKernelGGL(eigh_jacobi, dim3(1), dim3(kThreads), shmem, s, nt, reinterpret_cast<const double2 *>(cov),
                     evals, reinterpret_cast<double2 *>(evecs), info, max_sweeps);
  return hipGetLastError();
}

}  // namespace hh
