// C ABI of libhh: host-side validation, device-table cache, workspace layout and
// the ordered launch of the hot-path kernels.  No entry point waits for the
// device except the first-call table build of a configuration.
#include <algorithm>
#include <cmath>
#include <cstdarg>
#include <cstdio>
#include <cstring>
#include <map>
#include <mutex>
#include <new>
#include <string>
#include <tuple>
#include <vector>

#include "hh_internal.h"
#include "fourier.h"

namespace hh {

// ---------------------------------------------------------------- errors ----
static thread_local std::string g_err;

void set_error(const char *fmt, ...) {
  char buf[512];
  va_list ap;
  va_start(ap, fmt);
  vsnprintf(buf, sizeof buf, fmt, ap);
  va_end(ap);
  g_err = buf;
}

static hh_status fail(hh_status s, const char *fmt, ...) {
  char buf[512];
  va_list ap;
  va_start(ap, fmt);
  vsnprintf(buf, sizeof buf, fmt, ap);
  va_end(ap);
  g_err = buf;
  return s;
}

static hh_status device_fail(hipError_t e, const char *where) {
  return fail(HH_E_DEVICE, "%s: %s", where, hipGetErrorString(e));
}

// -------------------------------------------------------------- profiler ----
namespace {
struct ProfRec {
  std::string name;
  hipEvent_t a, b;
};
std::mutex g_prof_mu;
bool g_prof_on = false;
std::vector<ProfRec> g_prof;
std::vector<hipEvent_t> g_prof_pool;

hipEvent_t prof_event() {
  if (!g_prof_pool.empty()) {
    hipEvent_t e = g_prof_pool.back();
    g_prof_pool.pop_back();
    return e;
  }
  hipEvent_t e = nullptr;
  if (hipEventCreate(&e) != hipSuccess) return nullptr;
  return e;
}
}  // namespace

ProfScope::ProfScope(const char *n, hipStream_t s) : name(n), stream(s) {
  std::lock_guard<std::mutex> g(g_prof_mu);
  if (!g_prof_on) return;
  hipStreamCaptureStatus cs = hipStreamCaptureStatusNone;
  if (hipStreamIsCapturing(s, &cs) != hipSuccess || cs != hipStreamCaptureStatusNone) return;  // not in graphs
  hipEvent_t e = prof_event();
  if (e && hipEventRecord(e, s) == hipSuccess) ev0 = e;
}

ProfScope::~ProfScope() {
  if (!ev0) return;
  std::lock_guard<std::mutex> g(g_prof_mu);
  hipEvent_t e = prof_event();
  if (e && hipEventRecord(e, stream) == hipSuccess) g_prof.push_back({name, (hipEvent_t)ev0, e});
}

// ----------------------------------------------------------- plan cache ----
namespace {
using PlanKey = std::tuple<int, double, double, double, int, int>;
std::mutex g_plan_mu;
std::map<PlanKey, Plan> g_plans;
std::map<std::pair<int, int>, double *> g_dft;

bool is_pow2(int v) { return v > 0 && (v & (v - 1)) == 0; }

// exp(-i alpha (j - n/2)^2), phase formed from an exact integer square in FP64
std::vector<float2> chirp_table(int n, double alpha) {
  std::vector<float2> t(n);
  for (int j = 0; j < n; ++j) {
    const long long d = (long long)j - n / 2;
    const double ph = alpha * (double)(d * d);
    t[j] = make_float2((float)std::cos(ph), (float)-std::sin(ph));
  }
  return t;
}

// W_n^j = exp(-2 pi i j / n), from the exact rational angle j/n in FP64
std::vector<float2> twiddle_table(int n) {
  std::vector<float2> t(n);
  const double two_pi = 6.283185307179586476925286766559;
  for (int j = 0; j < n; ++j) {
    const double ang = two_pi * (double)j / (double)n;
    t[j] = make_float2((float)std::cos(ang), (float)-std::sin(ang));
  }
  return t;
}

hipError_t upload(float2 **dst, const std::vector<float2> &src) {
  hipError_t e = hipMalloc(dst, src.size() * sizeof(float2));
  if (e != hipSuccess) return e;
  return hipMemcpy(*dst, src.data(), src.size() * sizeof(float2), hipMemcpyHostToDevice);
}
}  // namespace

const Plan *get_plan(const hh_params &p) {
  int dev = 0;
  hipError_t e = hipGetDevice(&dev);
  if (e != hipSuccess) {
    set_error("hipGetDevice: %s", hipGetErrorString(e));
    return nullptr;
  }
  PlanKey key{dev, p.wavelength_m, p.distance_m, p.pitch_m, p.nx, p.ny};
  std::lock_guard<std::mutex> g(g_plan_mu);
  auto it = g_plans.find(key);
  if (it != g_plans.end()) return &it->second;
  const double alpha = M_PI * p.pitch_m * p.pitch_m / (p.wavelength_m * p.distance_m);
  Plan pl;
  pl.device = dev;
  pl.nx = p.nx;
  pl.ny = p.ny;
  int cus = 0;
  if (hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) == hipSuccess && cus > 0) pl.cus = cus;
  if ((e = upload(&pl.chirp_x, chirp_table(p.nx, alpha))) != hipSuccess ||
      (e = upload(&pl.chirp_y, chirp_table(p.ny, alpha))) != hipSuccess ||
      (e = upload(&pl.tw_x, twiddle_table(p.nx))) != hipSuccess ||
      (e = upload(&pl.tw_y, twiddle_table(p.ny))) != hipSuccess) {
    set_error("plan tables: %s", hipGetErrorString(e));
    (void)hipFree(pl.chirp_x);
    (void)hipFree(pl.chirp_y);
    (void)hipFree(pl.tw_x);
    (void)hipFree(pl.tw_y);
    return nullptr;
  }
  return &g_plans.emplace(key, pl).first->second;
}

const double *get_dft_basis(int nt) {
  int dev = 0;
  if (hipGetDevice(&dev) != hipSuccess) return nullptr;
  std::lock_guard<std::mutex> g(g_plan_mu);
  auto it = g_dft.find({dev, nt});
  if (it != g_dft.end()) return it->second;
  std::vector<double> w(2 * (size_t)nt * nt);
  const double two_pi = 6.283185307179586476925286766559, sc = 1.0 / std::sqrt((double)nt);
  for (int t = 0; t < nt; ++t)
    for (int f = 0; f < nt; ++f) {
      const long long tf = ((long long)t * f) % nt;  // exact reduction of the angle
      const double ang = two_pi * (double)tf / (double)nt;
      w[2 * ((size_t)t * nt + f)] = std::cos(ang) * sc;
      w[2 * ((size_t)t * nt + f) + 1] = -std::sin(ang) * sc;
    }
  double *d = nullptr;
  if (hipMalloc(&d, w.size() * sizeof(double)) != hipSuccess) return nullptr;
  if (hipMemcpy(d, w.data(), w.size() * sizeof(double), hipMemcpyHostToDevice) != hipSuccess) {
    (void)hipFree(d);
    return nullptr;
  }
  g_dft[{dev, nt}] = d;
  return d;
}

// ------------------------------------------------------------ validation ----
namespace {
hh_status check_optics(const hh_params *p) {
  if (!p) return fail(HH_E_INVALID, "params is NULL");
  if (!(std::isfinite(p->wavelength_m) && p->wavelength_m > 0))
    return fail(HH_E_INVALID, "wavelength_m must be finite and > 0");
  if (!(std::isfinite(p->distance_m) && p->distance_m != 0))
    return fail(HH_E_INVALID, "distance_m must be finite and != 0");
  if (!(std::isfinite(p->pitch_m) && p->pitch_m > 0)) return fail(HH_E_INVALID, "pitch_m must be finite and > 0");
  return HH_OK;
}

hh_status check_shape(const hh_params *p) {
  if (!p) return fail(HH_E_INVALID, "params is NULL");
  if (p->nx <= 0 || p->ny <= 0) return fail(HH_E_INVALID, "nx, ny must be > 0");
  if (!is_pow2(p->nx) || !is_pow2(p->ny) || p->nx < 8 || p->ny < 8 || p->nx > 4096 || p->ny > 4096)
    return fail(HH_E_UNSUPPORTED, "nx=%d ny=%d: frame sides must be powers of two in [8, 4096]", p->nx, p->ny);
  if (p->eigh_solver != HH_EIGH_TRIDIAG && p->eigh_solver != HH_EIGH_JACOBI)
    return fail(HH_E_INVALID, "eigh_solver=%d unknown", p->eigh_solver);
  return HH_OK;
}

hh_status check_stack(const hh_params *p) {
  hh_status s = check_shape(p);
  if (s) return s;
  if (p->nt < 2 || p->nt > 64) return fail(HH_E_UNSUPPORTED, "nt=%d: stack length must be in [2, 64]", p->nt);
  return HH_OK;
}

hh_status check_select(const hh_params *p) {
  if (!(0 <= p->k_lo && p->k_lo <= p->k_hi && p->k_hi < p->nt))
    return fail(HH_E_INVALID, "kept range k_lo=%d k_hi=%d must satisfy 0 <= k_lo <= k_hi < nt=%d", p->k_lo,
                p->k_hi, p->nt);
  if (p->proj_mode < HH_PROJ_AUTO || p->proj_mode > HH_PROJ_FIRST)
    return fail(HH_E_INVALID, "proj_mode=%d unknown", p->proj_mode);
  return HH_OK;
}

// from_frames: the entry point starts from frames (hh_pipeline and the batched
// forms); the FP16 storage form exists only there.
hh_status check_precision(const hh_params *p, bool from_frames) {
  if (p->precision < HH_FP32 || p->precision > HH_EXACT)
    return fail(HH_E_INVALID, "precision=%d unknown", p->precision);
  if (p->precision != HH_FP32 && p->precision != HH_EXACT && p->nt > 32)
    return fail(HH_E_UNSUPPORTED, "precision form %d is built for nt <= 32 (nt=%d)", p->precision, p->nt);
  if ((p->precision == HH_FP16_STORE || p->precision == HH_EXACT) && !from_frames)
    return fail(HH_E_UNSUPPORTED, "precision form %d applies to entry points that start from frames", p->precision);
  if (p->proj_mode == HH_PROJ_FIRST && !from_frames)
    return fail(HH_E_UNSUPPORTED, "HH_PROJ_FIRST applies to entry points that start from frames");
  if (p->proj_mode == HH_PROJ_FIRST && p->precision != HH_EXACT)
    return fail(HH_E_INVALID, "HH_PROJ_FIRST needs precision HH_EXACT (covariance from the frames)");
  return HH_OK;
}

// the image-from-holograms entry points take every projection mode but HH_PROJ_FIRST
hh_status check_holo_proj(const hh_params *p) {
  if (p->proj_mode == HH_PROJ_FIRST)
    return fail(HH_E_UNSUPPORTED, "HH_PROJ_FIRST starts from frames (hh_project_frames, hh_pipeline)");
  return HH_OK;
}

// alignment the frames of one stack need under p's form
size_t frames_align(const hh_params &) { return 16; }  // 16-byte loads of 8 pixels

bool aligned(const void *ptr, size_t a) { return ((uintptr_t)ptr % a) == 0; }

// ------------------------------------------------------------ tuning ----
// Launch choices per problem shape, filled by hh_autotune or hh_tuning_set:
// FFT shapes and the group size per (device, nx, ny); the covariance split-K
// chunk per (device, nx*ny, nt, precision).  Absent entries use the defaults.
using FftKey = std::tuple<int, int, int>;
using GramKey = std::tuple<int, long long, int, int>;
std::mutex g_tune_mu;
std::map<FftKey, Tune> g_fft_tune;
std::map<GramKey, std::pair<int, int>> g_gram_tune;  // (pixels per wave, reference of the split)

int current_device() {
  int d = 0;
  return hipGetDevice(&d) == hipSuccess ? d : -1;
}

Tune get_tune(const hh_params &p) {
  const int d = current_device();
  std::lock_guard<std::mutex> g(g_tune_mu);
  Tune t;
  auto f = g_fft_tune.find(FftKey{d, p.nx, p.ny});
  if (f != g_fft_tune.end()) t = f->second;
  auto q = g_gram_tune.find(GramKey{d, (long long)p.nx * p.ny, p.nt, p.precision});
  t.pxw = q != g_gram_tune.end() ? q->second.first : kGramPxwMin;
  t.gram_ref = q != g_gram_tune.end() ? q->second.second : 0;
  return t;
}

void put_tune(const hh_params &p, const Tune &t) {
  const int d = current_device();
  std::lock_guard<std::mutex> g(g_tune_mu);
  g_fft_tune[FftKey{d, p.nx, p.ny}] = t;
  g_gram_tune[GramKey{d, (long long)p.nx * p.ny, p.nt, p.precision}] = {t.pxw, t.gram_ref};
}

int default_group(const hh_params &p) { return fresnel_group_frames(p.nx, p.ny, 1 << 30, 0); }

hh_status check_tune(const hh_params &p, const hh_tuning &t) {
  const int nrows = p.nx >= 512 ? 10 : 1, ncols = p.ny >= 512 ? 8 : 1;
  if (t.fft_rows < 0 || t.fft_rows >= nrows) return fail(HH_E_INVALID, "fft_rows=%d: %d shape(s) at nx=%d", t.fft_rows, nrows, p.nx);
  if (t.fft_cols < 0 || t.fft_cols >= ncols) return fail(HH_E_INVALID, "fft_cols=%d: %d shape(s) at ny=%d", t.fft_cols, ncols, p.ny);
  if (t.gram_pxw != 256 && t.gram_pxw != 512 && t.gram_pxw != 1024)
    return fail(HH_E_INVALID, "gram_pxw=%d: must be 256, 512 or 1024", t.gram_pxw);
  if (t.gram_ref < 0 || t.gram_ref > 1) return fail(HH_E_INVALID, "gram_ref=%d: must be 0 or 1", t.gram_ref);
  if (t.fused < 0 || t.fused > 1) return fail(HH_E_INVALID, "fused=%d: must be 0 or 1", t.fused);
  if (t.group < 0 || t.group > 4 * default_group(p))
    return fail(HH_E_INVALID, "group=%d: must be in [0, %d] (0 = default)", t.group, 4 * default_group(p));
  return HH_OK;
}

struct PipeLayout {
  GramLayout g;
  bool r16 = false;    // FP16 storage form
  bool first = false;  // projection first: the hologram area holds the K row-transformed components
  size_t holo = 0, r16buf = 0, group = 0, mean = 0, m = 0, eparts = 0;
  size_t part = 0, part2 = 0, cov = 0, evals = 0, evecs = 0, info = 0, total = 0;
};

// with_holo = false: the layout of steps (b)-(e) on a hologram stack the caller holds
PipeLayout pipe_layout(const hh_params *p, bool with_holo = true) {
  PipeLayout L;
  const long long npix = (long long)p->nx * p->ny;
  L.g = gram_layout(p->nt, npix);
  L.r16 = with_holo && p->precision == HH_FP16_STORE;
  size_t o = 0;
  if (L.r16) {
    L.r16buf = o; o = align_up(o + (size_t)p->nt * npix * sizeof(h2));
    L.group = o; o = align_up(o + (size_t)fresnel_group_frames(p->nx, p->ny, p->nt, 0) * npix * sizeof(float2));
    L.mean = o; o = align_up(o + (size_t)npix * sizeof(float));
    L.m = o; o = align_up(o + (size_t)npix * sizeof(float2));
  } else {
    L.holo = o;
    if (with_holo) o = align_up(o + (size_t)p->nt * npix * sizeof(float2));
  }
  L.first = with_holo && p->proj_mode == HH_PROJ_FIRST;
  if (L.first) {
    L.eparts = o;
    o = align_up(o + (size_t)kMaxEnergyChunks * npix * sizeof(float));
  }
  L.part = o; o = align_up(o + L.g.partial_bytes);
  L.part2 = o; o = align_up(o + L.g.partial2_bytes);
  L.cov = o; o = align_up(o + (size_t)p->nt * p->nt * 2 * sizeof(double));
  L.evals = o; o = align_up(o + (size_t)p->nt * sizeof(double));
  L.evecs = o; o = align_up(o + (size_t)p->nt * p->nt * 2 * sizeof(double));
  L.info = o; o = align_up(o + sizeof(int));
  L.total = o;
  return L;
}

// Power-of-two scale of the stored FP16 residual: |frame - mean| <= 65535, so
// |R[p]| <= npix * 65535 and npix * 65535 * s stays below the FP16 maximum 65504.
float r16_inv_scale(long long npix) {
  int e = 1;
  while ((1ll << (e - 1)) < npix) ++e;  // 2^(e-1) >= npix, npix a power of two
  return std::ldexp(1.0f, e);             // 1 / s = 2 npix
}

// Steps (a)+(b) of one stack in its workspace region (frames given), or step (b)
// on the caller's hologram (holo given).  Fills the views that steps (d)+(e) read.
struct StackViews {
  const float2 *H = nullptr;
  const float2 *T = nullptr;  // three-pass FP32 form: the column-transformed frames (not H)
  const h2 *r16 = nullptr;
  const float2 *m = nullptr;
  float inv_s = 1.f;
  double *cov = nullptr;
  const double *part2 = nullptr;  // covariance partials the eigensolver assembles into cov
  int g2 = 0, D = 0;
  // projection first: the frames, the component and partial-image areas, the plan's tables
  const uint16_t *frames = nullptr;
  float2 *inter = nullptr;
  float *eparts = nullptr;
  const Plan *pl = nullptr;
};

hipError_t enqueue_front(const hh_params &p, const Plan *pl, const PipeLayout &L, char *ws, const uint16_t *frames,
                         const float2 *holo, StackViews &v, hipStream_t s) {
  const long long npix = (long long)p.nx * p.ny;
  const Tune tu = get_tune(p);
  GramLayout gl = gram_layout(p.nt, npix, tu.pxw);  // offsets in L are sized for the smallest chunk
  gl.ref = tu.gram_ref;
  double *part = reinterpret_cast<double *>(ws + L.part), *part2 = reinterpret_cast<double *>(ws + L.part2);
  v.cov = reinterpret_cast<double *>(ws + L.cov);
  v.part2 = part2;
  v.g2 = gl.groups2;
  v.D = gl.D;
  if (L.r16) {
    h2 *r = reinterpret_cast<h2 *>(ws + L.r16buf);
    float2 *m = reinterpret_cast<float2 *>(ws + L.m);
    v.inv_s = r16_inv_scale(npix);
    v.r16 = r;
    v.m = m;
    hipError_t e = launch_fresnel_r16(*pl, tu, frames, p.nt, reinterpret_cast<float *>(ws + L.mean), m,
                                      reinterpret_cast<float2 *>(ws + L.group), r, 1.0f / v.inv_s, s);
    if (e != hipSuccess) return e;
    return launch_gram_r16(gl, r, m, p.nt, npix, v.inv_s, part, part2, v.cov, s, false);
  }
  if (L.first) {  // C from the frames; the transforms wait for V
    v.frames = frames;
    v.inter = reinterpret_cast<float2 *>(ws + L.holo);
    v.eparts = reinterpret_cast<float *>(ws + L.eparts);
    v.pl = pl;
    return launch_gram_u16(gl, frames, p.nt, npix, part, part2, v.cov, s, false);
  }
  if (frames && p.precision == HH_FP32 && tu.fused && fused_supported(p.nx, p.ny, p.nt)) {
    float2 *Tb = reinterpret_cast<float2 *>(ws + L.holo);
    int groups = 0;
    hipError_t e = launch_fused_front(*pl, frames, p.nt, Tb, L.g.groups, part, &groups, s);
    if (e != hipSuccess) return e;
    GramLayout fl = gl;
    fl.groups = groups;
    fl.groups2 = groups < fl.groups2 ? groups : fl.groups2;
    v.T = Tb;
    v.pl = pl;
    v.g2 = fl.groups2;
    return launch_gram_tail(fl, p.nt, part, part2, v.cov, s, false);
  }
  if (frames) {
    float2 *H = reinterpret_cast<float2 *>(ws + L.holo);
    hipError_t e = launch_fresnel(*pl, tu, frames, p.nt, H, s);
    if (e != hipSuccess) return e;
    v.H = H;
    if (p.precision == HH_EXACT) return launch_gram_u16(gl, frames, p.nt, npix, part, part2, v.cov, s, false);
  } else {
    v.H = holo;
  }
  return launch_gram(gl, v.H, p.nt, npix, part, part2, v.cov, s, p.precision, false);
}

hipError_t enqueue_back(const hh_params &p, const StackViews &v, const double *V, float *image, hipStream_t s) {
  const long long npix = (long long)p.nx * p.ny;
  if (v.T) return launch_fused_back(*v.pl, v.T, p.nt, V, p.k_lo, p.k_hi, p.proj_mode, image, s);
  // C = N_pix I^T I is real symmetric, so the solver's eigenvectors are real: Re V suffices
  if (v.inter)
    return launch_project_frames(*v.pl, v.frames, p.nt, V, p.k_lo, p.k_hi, true, v.inter, v.eparts, image, s);
  if (v.r16) return launch_project_r16(v.r16, v.m, v.inv_s, p.nt, npix, V, p.k_lo, p.k_hi, p.proj_mode, image, s);
  return launch_project(v.H, p.nt, npix, V, p.k_lo, p.k_hi, p.proj_mode, image, s, p.precision);
}

constexpr int kMaxBatch = 4096;

// One stack of a batch: either frames (steps (a)-(e)) or a hologram stack (steps (b)-(e)).
struct BatchItem {
  const uint16_t *frames;
  const float2 *holo;
  float *image;
  double *evals, *evecs;
  int32_t *info;
};

size_t batch_ws_bytes(const hh_params *p, int32_t n, bool with_holo) {
  if (!p || n < 1 || n > kMaxBatch) return 0;
  size_t total = 0;
  for (int i = 0; i < n; ++i) {
    if (check_stack(p + i) || check_select(p + i) || (with_holo && check_optics(p + i))) return 0;
    total += align_up(pipe_layout(p + i, with_holo).total);
  }
  return total;
}

// Stacks whose eigenproblems go first in the captured form: those of the largest
// solver class present (n > 32, then n > 16); when every stack is in that class,
// the first half.
std::vector<int> early_stacks(const hh_params *p, int n) {
  std::vector<int> first;
  int top = 0;
  for (int i = 0; i < n; ++i) top = std::max(top, p[i].nt > 32 ? 2 : p[i].nt > 16 ? 1 : 0);
  for (int i = 0; i < n; ++i)
    if ((p[i].nt > 32 ? 2 : p[i].nt > 16 ? 1 : 0) == top) first.push_back(i);
  if ((int)first.size() == n) first.resize((n + 1) / 2);
  return first;
}

// Validates every item, then enqueues.
// Without a branch (eager calls: a caller overlaps batches on streams of its own):
// on s, every stack's transform and covariance, one eigensolver launch per solver
// class, then every projection.
// With a branch stream (the captured form): on s, the transforms and covariances of
// the early stacks (early_stacks); then on the branch, which waits for them, their
// eigenproblems (one launch per solver class) and projections, while s goes on with
// the transforms, covariances, eigenproblems and projections of the other stacks;
// s finally waits for the branch.  The eigensolver is one workgroup per problem and
// latency-bound, so its run on the branch overlaps the bandwidth-bound work of the
// other stacks.  (One branch: with more, the graph runtime placed later transforms
// in the hardware queue behind a branch's long solve.)  Each stack's results do not
// depend on the schedule.
hh_status run_batch(const hh_params *p, int n, const BatchItem *it, void *workspace, size_t ws_bytes, hipStream_t s,
                    const char *who, hipStream_t branch = nullptr) {
  const bool with_holo = it[0].frames != nullptr;
  size_t need = 0;
  for (int i = 0; i < n; ++i) {
    hh_status st;
    if ((with_holo && (st = check_optics(p + i))) || (st = check_stack(p + i)) || (st = check_select(p + i)) ||
        (st = check_precision(p + i, with_holo))) {
      const std::string msg = g_err;
      return fail(st, "stack %d: %s", i, msg.c_str());
    }
    if (!it[i].image) return fail(HH_E_INVALID, "stack %d: image must be non-NULL", i);
    if ((it[i].frames && !aligned(it[i].frames, frames_align(p[i]))) ||
        !aligned(it[i].image, 8) || (it[i].evals && !aligned(it[i].evals, 8)) ||
        (it[i].evecs && !aligned(it[i].evecs, 16)) || (it[i].info && !aligned(it[i].info, 4)))
      return fail(HH_E_INVALID, "stack %d: arrays misaligned", i);
    need += align_up(pipe_layout(p + i, with_holo).total);
  }
  if (!workspace || ws_bytes < need || !aligned(workspace, 256))
    return fail(HH_E_WORKSPACE, "%s workspace: need %zu bytes (256-byte aligned), got %zu", who, need, ws_bytes);
  std::vector<const Plan *> plans(n, nullptr);
  if (with_holo)
    for (int i = 0; i < n; ++i)
      if (!(plans[i] = get_plan(p[i]))) return HH_E_DEVICE;
  std::vector<EighProblem> probs(n);
  std::vector<StackViews> views(n);
  std::vector<size_t> offs(n);
  {
    size_t o = 0;
    for (int i = 0; i < n; ++i) {
      offs[i] = o;
      o += align_up(pipe_layout(p + i, with_holo).total);
    }
  }
  char *ws0 = static_cast<char *>(workspace);
  auto front = [&](int i) {
    const PipeLayout L = pipe_layout(p + i, with_holo);
    char *ws = ws0 + offs[i];
    const hipError_t e = enqueue_front(p[i], plans[i], L, ws, it[i].frames, it[i].holo, views[i], s);
    probs[i] = EighProblem{p[i].nt,
                           views[i].cov,
                           it[i].evals ? it[i].evals : reinterpret_cast<double *>(ws + L.evals),
                           it[i].evecs ? it[i].evecs : reinterpret_cast<double *>(ws + L.evecs),
                           it[i].info ? it[i].info : reinterpret_cast<int *>(ws + L.info),
                           views[i].part2,
                           views[i].g2,
                           views[i].D,
                           p[i].eigh_solver};
    return e;
  };
  auto back = [&](const std::vector<int> &set, hipStream_t st) {
    std::vector<EighProblem> sub;
    for (int i : set) sub.push_back(probs[i]);
    hipError_t e = sub.empty() ? hipSuccess : launch_eigh_batch(sub.data(), (int)sub.size(), 40, st);
    for (size_t k = 0; k < set.size() && e == hipSuccess; ++k)
      e = enqueue_back(p[set[k]], views[set[k]], probs[set[k]].evecs, it[set[k]].image, st);
    return e;
  };

  hipError_t e = hipSuccess;
  if (!branch || n < 2) {
    std::vector<int> all(n);
    for (int i = 0; i < n; ++i) all[i] = i;
    for (int i = 0; i < n && e == hipSuccess; ++i) e = front(i);
    if (e == hipSuccess) e = back(all, s);
    if (e != hipSuccess) return device_fail(e, who);
    return HH_OK;
  }
  const std::vector<int> early = early_stacks(p, n);
  std::vector<char> is_early(n, 0);
  for (int i : early) is_early[i] = 1;
  std::vector<int> late;
  for (int i = 0; i < n; ++i)
    if (!is_early[i]) late.push_back(i);
  hipEvent_t fork = nullptr, join = nullptr;
  if ((e = hipEventCreateWithFlags(&fork, hipEventDisableTiming)) != hipSuccess) return device_fail(e, who);
  if ((e = hipEventCreateWithFlags(&join, hipEventDisableTiming)) != hipSuccess) {
    (void)hipEventDestroy(fork);
    return device_fail(e, who);
  }
  for (size_t k = 0; k < early.size() && e == hipSuccess; ++k) e = front(early[k]);
  bool forked = false;
  if (e == hipSuccess) e = hipEventRecord(fork, s);
  if (e == hipSuccess) e = hipStreamWaitEvent(branch, fork, 0);
  if (e == hipSuccess) {
    forked = true;
    e = back(early, branch);
  }
  for (size_t k = 0; k < late.size() && e == hipSuccess; ++k) e = front(late[k]);
  if (e == hipSuccess) e = back(late, s);
  // the join is enqueued whenever the fork was, so that a capture ends joined
  if (forked) {
    hipError_t ej = hipEventRecord(join, branch);
    if (ej == hipSuccess) ej = hipStreamWaitEvent(s, join, 0);
    if (e == hipSuccess) e = ej;
  }
  (void)hipEventDestroy(fork);
  (void)hipEventDestroy(join);
  if (e != hipSuccess) return device_fail(e, who);
  return HH_OK;
}

size_t cov_ws_bytes(const hh_params *p) {
  const GramLayout g = gram_layout(p->nt, (long long)p->nx * p->ny);
  return align_up(g.partial_bytes) + align_up(g.partial2_bytes);
}
}  // namespace

}  // namespace hh

using namespace hh;

extern "C" {

const char *hh_status_string(hh_status s) {
  switch (s) {
    case HH_OK: return "ok";
    case HH_E_INVALID: return "invalid argument";
    case HH_E_UNSUPPORTED: return "unsupported";
    case HH_E_WORKSPACE: return "workspace too small";
    case HH_E_DEVICE: return "device error";
    case HH_E_NOT_CONVERGED: return "eigensolver did not converge";
  }
  return "unknown status";
}

const char *hh_last_error(void) { return g_err.c_str(); }

size_t hh_workspace_bytes(const hh_params *p) {
  if (check_optics(p) || check_stack(p) || check_select(p)) return 0;
  return pipe_layout(p).total;
}

size_t hh_covariance_workspace_bytes(const hh_params *p) {
  if (check_stack(p)) return 0;
  return cov_ws_bytes(p);
}

hh_status hh_fresnel(const hh_params *p, const uint16_t *frames, int32_t nframes, float *holo, void *stream) {
  hh_status st;
  if ((st = check_optics(p)) || (st = check_shape(p))) return st;
  if (nframes < 0 || nframes > 65535) return fail(HH_E_INVALID, "nframes=%d must be in [0, 65535]", nframes);
  if (nframes == 0) return HH_OK;
  if (!frames || !holo) return fail(HH_E_INVALID, "frames and holo must be non-NULL");
  if (!aligned(frames, 16) || !aligned(holo, 16)) return fail(HH_E_INVALID, "frames/holo must be 16-byte aligned");
  const Plan *pl = get_plan(*p);
  if (!pl) return HH_E_DEVICE;
  hipError_t e =
      launch_fresnel(*pl, get_tune(*p), frames, nframes, reinterpret_cast<float2 *>(holo), (hipStream_t)stream);
  if (e != hipSuccess) return device_fail(e, "hh_fresnel");
  return HH_OK;
}

hh_status hh_covariance(const hh_params *p, const float *holo, double *cov, void *workspace, size_t ws_bytes,
                        void *stream) {
  hh_status st;
  if ((st = check_stack(p)) || (st = check_precision(p, false))) return st;
  if (!holo || !cov) return fail(HH_E_INVALID, "holo and cov must be non-NULL");
  if (!aligned(holo, 16) || !aligned(cov, 16)) return fail(HH_E_INVALID, "holo/cov misaligned");
  const size_t need = cov_ws_bytes(p);
  if (!workspace || ws_bytes < need || !aligned(workspace, 256))
    return fail(HH_E_WORKSPACE, "covariance workspace: need %zu bytes (256-byte aligned), got %zu", need, ws_bytes);
  const long long npix = (long long)p->nx * p->ny;
  const GramLayout g = gram_layout(p->nt, npix);                     // sizes the workspace
  GramLayout gl = gram_layout(p->nt, npix, get_tune(*p).pxw);  // the launch
  gl.ref = get_tune(*p).gram_ref;
  char *ws = static_cast<char *>(workspace);
  hipError_t e = launch_gram(gl, reinterpret_cast<const float2 *>(holo), p->nt, npix, reinterpret_cast<double *>(ws),
                             reinterpret_cast<double *>(ws + align_up(g.partial_bytes)), cov, (hipStream_t)stream,
                             p->precision);
  if (e != hipSuccess) return device_fail(e, "hh_covariance");
  return HH_OK;
}

// ------------------------------------------------------- allocation-free ----
// Device scratch of hh_covariance_noalloc: the covariance's split-K partials.  One
// copy per GPU, held until the process ends.  Host code never uses the array's name
// as an address: each device's copy is looked up once with hipGetSymbolAddress and
// that pointer is what the kernels receive.
constexpr size_t kNoAllocScratchBytes = size_t(48) << 20;
static __device__ __align__(256) char scratch[kNoAllocScratchBytes];

namespace {
std::mutex g_scratch_mu;
std::map<int, char *> g_scratch_ptr;  // device -> address of that device's scratch

// The current device's scratch address (looked up on its first use on that device).
hh_status scratch_ptr(char **out) {
  const int dev = current_device();
  if (dev < 0) return fail(HH_E_DEVICE, "hh_covariance_noalloc: no current HIP device");
  std::lock_guard<std::mutex> g(g_scratch_mu);
  auto it = g_scratch_ptr.find(dev);
  if (it == g_scratch_ptr.end()) {
    void *ptr = nullptr;
    const hipError_t e = hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch));
    if (e != hipSuccess || !ptr) return device_fail(e != hipSuccess ? e : hipErrorInvalidSymbol, "hipGetSymbolAddress");
    it = g_scratch_ptr.emplace(dev, static_cast<char *>(ptr)).first;
  }
  *out = it->second;
  return HH_OK;
}
}  // namespace

size_t hh_covariance_noalloc_max_bytes(void) { return kNoAllocScratchBytes; }

hh_status hh_covariance_noalloc(const hh_params *p, const float *holo, double *cov, void *stream) {
  hh_status st;
  if ((st = check_stack(p)) || (st = check_precision(p, false))) return st;
  if (!holo || !cov) return fail(HH_E_INVALID, "holo and cov must be non-NULL");
  if (!aligned(holo, 16) || !aligned(cov, 16)) return fail(HH_E_INVALID, "holo/cov misaligned");
  const long long npix = (long long)p->nx * p->ny;
  // the same launch as hh_covariance: the same split-K chunk and reference
  GramLayout gl = gram_layout(p->nt, npix, get_tune(*p).pxw);
  gl.ref = get_tune(*p).gram_ref;
  const size_t need = align_up(gl.partial_bytes) + align_up(gl.partial2_bytes);
  if (need > kNoAllocScratchBytes)
    return fail(HH_E_UNSUPPORTED,
                "hh_covariance_noalloc: nt=%d, %lld pixels at %d-pixel chunks need %zu bytes of scratch; the "
                "static scratch holds %zu (use hh_covariance with a workspace)",
                p->nt, npix, gl.pxw, need, kNoAllocScratchBytes);
  char *ws = nullptr;
  if ((st = scratch_ptr(&ws))) return st;
  hipError_t e = launch_gram(gl, reinterpret_cast<const float2 *>(holo), p->nt, npix, reinterpret_cast<double *>(ws),
                             reinterpret_cast<double *>(ws + align_up(gl.partial_bytes)), cov, (hipStream_t)stream,
                             p->precision);
  if (e != hipSuccess) return device_fail(e, "hh_covariance_noalloc");
  return HH_OK;
}

hh_status hh_covariance_frames(const hh_params *p, const uint16_t *frames, double *cov, void *workspace,
                               size_t ws_bytes, void *stream) {
  hh_status st;
  if ((st = check_stack(p))) return st;
  if (!frames || !cov) return fail(HH_E_INVALID, "frames and cov must be non-NULL");
  if (!aligned(frames, 16) || !aligned(cov, 16)) return fail(HH_E_INVALID, "frames/cov must be 16-byte aligned");
  const size_t need = cov_ws_bytes(p);
  if (!workspace || ws_bytes < need || !aligned(workspace, 256))
    return fail(HH_E_WORKSPACE, "covariance workspace: need %zu bytes (256-byte aligned), got %zu", need, ws_bytes);
  const long long npix = (long long)p->nx * p->ny;
  const GramLayout g = gram_layout(p->nt, npix);
  hh_params q = *p;
  q.precision = HH_EXACT;
  const GramLayout gl = gram_layout(p->nt, npix, get_tune(q).pxw);
  char *ws = static_cast<char *>(workspace);
  hipError_t e = launch_gram_u16(gl, frames, p->nt, npix, reinterpret_cast<double *>(ws),
                                 reinterpret_cast<double *>(ws + align_up(g.partial_bytes)), cov, (hipStream_t)stream);
  if (e != hipSuccess) return device_fail(e, "hh_covariance_frames");
  return HH_OK;
}

hh_status hh_eigh_ex(int32_t nt, const double *cov, double *evals, double *evecs, int32_t *info, int32_t max_sweeps,
                     void *stream) {
  if (nt < 2 || nt > 64) return fail(HH_E_UNSUPPORTED, "nt=%d: must be in [2, 64]", nt);
  if (!cov || !evals || !evecs || !info) return fail(HH_E_INVALID, "cov, evals, evecs, info must be non-NULL");
  if (!aligned(cov, 16) || !aligned(evecs, 16) || !aligned(evals, 8) || !aligned(info, 4))
    return fail(HH_E_INVALID, "eigh arrays misaligned");
  if (max_sweeps < 0) return fail(HH_E_INVALID, "max_sweeps must be >= 0");
  hipError_t e = launch_eigh(nt, cov, evals, evecs, info, max_sweeps, (hipStream_t)stream);
  if (e != hipSuccess) return device_fail(e, "hh_eigh");
  return HH_OK;
}

hh_status hh_eigh_tridiag(int32_t nt, const double *cov, double *evals, double *evecs, int32_t *info,
                          int32_t max_iter, void *stream) {
  if (nt < 2 || nt > 64) return fail(HH_E_UNSUPPORTED, "nt=%d: must be in [2, 64]", nt);
  if (!cov || !evals || !evecs || !info) return fail(HH_E_INVALID, "cov, evals, evecs, info must be non-NULL");
  if (!aligned(cov, 16) || !aligned(evecs, 16) || !aligned(evals, 8) || !aligned(info, 4))
    return fail(HH_E_INVALID, "eigh arrays misaligned");
  if (max_iter < 0) return fail(HH_E_INVALID, "max_iter must be >= 0");
  EighProblem prob{nt, cov, evals, evecs, info};
  prob.method = HH_EIGH_TRIDIAG;
  hipError_t e = launch_eigh_batch(&prob, 1, max_iter, (hipStream_t)stream);
  if (e != hipSuccess) return device_fail(e, "hh_eigh_tridiag");
  return HH_OK;
}

hh_status hh_eigh(int32_t nt, const double *cov, double *evals, double *evecs, int32_t *info, void *stream) {
  return hh_eigh_ex(nt, cov, evals, evecs, info, 40, stream);
}

hh_status hh_svd_filter(const hh_params *p, const float *holo, const double *evecs, float *out, void *stream) {
  hh_status st;
  if ((st = check_stack(p)) || (st = check_select(p)) || (st = check_holo_proj(p))) return st;
  if (!holo || !evecs || !out) return fail(HH_E_INVALID, "holo, evecs, out must be non-NULL");
  if (!aligned(holo, 16) || !aligned(evecs, 16) || !aligned(out, 16))
    return fail(HH_E_INVALID, "holo/evecs/out must be 16-byte aligned");
  const size_t bytes = (size_t)p->nt * p->nx * p->ny * sizeof(float2);
  const char *h0 = reinterpret_cast<const char *>(holo), *o0 = reinterpret_cast<const char *>(out);
  if (h0 < o0 + bytes && o0 < h0 + bytes) return fail(HH_E_INVALID, "out must not overlap holo");
  hipError_t e = launch_svd_filter(reinterpret_cast<const float2 *>(holo), p->nt, (long long)p->nx * p->ny, evecs,
                                   p->k_lo, p->k_hi, p->proj_mode, reinterpret_cast<float2 *>(out),
                                   (hipStream_t)stream);
  if (e != hipSuccess) return device_fail(e, "hh_svd_filter");
  return HH_OK;
}

hh_status hh_project_render(const hh_params *p, const float *holo, const double *evecs, float *image, void *stream) {
  hh_status st;
  if ((st = check_stack(p)) || (st = check_select(p)) || (st = check_precision(p, false))) return st;
  if (!holo || !evecs || !image) return fail(HH_E_INVALID, "holo, evecs, image must be non-NULL");
  if (!aligned(holo, 16) || !aligned(evecs, 16) || !aligned(image, 8))
    return fail(HH_E_INVALID, "holo/evecs/image misaligned");
  hipError_t e = launch_project(reinterpret_cast<const float2 *>(holo), p->nt, (long long)p->nx * p->ny, evecs,
                                p->k_lo, p->k_hi, p->proj_mode, image, (hipStream_t)stream, p->precision);
  if (e != hipSuccess) return device_fail(e, "hh_project_render");
  return HH_OK;
}

size_t hh_project_frames_workspace_bytes(const hh_params *p) {
  if (check_stack(p) || check_select(p)) return 0;
  const long long npix = (long long)p->nx * p->ny;
  const int K = p->k_hi - p->k_lo + 1;
  return align_up((size_t)K * npix * sizeof(float2)) + align_up((size_t)kMaxEnergyChunks * npix * sizeof(float));
}

hh_status hh_project_frames(const hh_params *p, const uint16_t *frames, const double *evecs, float *image,
                            void *workspace, size_t ws_bytes, void *stream) {
  hh_status st;
  if ((st = check_optics(p)) || (st = check_stack(p)) || (st = check_select(p))) return st;
  if (!frames || !evecs || !image) return fail(HH_E_INVALID, "frames, evecs, image must be non-NULL");
  if (!aligned(frames, 16) || !aligned(evecs, 16) || !aligned(image, 8))
    return fail(HH_E_INVALID, "frames/evecs/image misaligned");
  const size_t need = hh_project_frames_workspace_bytes(p);
  if (!workspace || ws_bytes < need || !aligned(workspace, 256))
    return fail(HH_E_WORKSPACE, "projection workspace: need %zu bytes (256-byte aligned), got %zu", need, ws_bytes);
  const Plan *pl = get_plan(*p);
  if (!pl) return HH_E_DEVICE;
  const long long npix = (long long)p->nx * p->ny;
  const int K = p->k_hi - p->k_lo + 1;
  char *ws = static_cast<char *>(workspace);
  hipError_t e = launch_project_frames(*pl, frames, p->nt, evecs, p->k_lo, p->k_hi, false,
                                       reinterpret_cast<float2 *>(ws),
                                       reinterpret_cast<float *>(ws + align_up((size_t)K * npix * sizeof(float2))),
                                       image, (hipStream_t)stream);
  if (e != hipSuccess) return device_fail(e, "hh_project_frames");
  return HH_OK;
}

namespace {
// Fourier demodulation of nwin windows w of the frames holo[w hop .. w hop + nt - 1].
hh_status fourier_windows(const hh_params *p, const float *holo, int nwin, int hop, float *images, void *stream,
                          const char *who) {
  hh_status st;
  if ((st = check_stack(p)) || (st = check_select(p)) || (st = check_holo_proj(p))) return st;
  if (!holo || !images) return fail(HH_E_INVALID, "holo, images must be non-NULL");
  if (!aligned(holo, 16) || !aligned(images, 8)) return fail(HH_E_INVALID, "holo/images misaligned");
  if (nwin < 1 || nwin > 4096 || hop < 1 || hop > 4096)
    return fail(HH_E_INVALID, "nwin=%d hop=%d: must be in [1, 4096]", nwin, hop);
  const long long npix = (long long)p->nx * p->ny;
  hipError_t e = hipSuccess;
  if (fourier_band_supported(p->nt)) {
    // a power-of-two n_t: every pixel's DFT along t in registers
    e = launch_fourier_band(reinterpret_cast<const float2 *>(holo), p->nt, npix, nwin, hop, p->k_lo, p->k_hi, images,
                            (hipStream_t)stream);
  } else {
    // any other n_t: the projection onto the band's DFT basis columns, window by window
    const double *W = get_dft_basis(p->nt);
    if (!W) return fail(HH_E_DEVICE, "DFT basis upload failed");
    for (int w = 0; w < nwin && e == hipSuccess; ++w)
      e = launch_project(reinterpret_cast<const float2 *>(holo) + (long long)w * hop * npix, p->nt, npix, W, p->k_lo,
                         p->k_hi, p->proj_mode, images + (long long)w * npix, (hipStream_t)stream);
  }
  if (e != hipSuccess) return device_fail(e, who);
  return HH_OK;
}
}  // namespace

hh_status hh_fourier_render(const hh_params *p, const float *holo, float *image, void *stream) {
  return fourier_windows(p, holo, 1, 1, image, stream, "hh_fourier_render");
}

hh_status hh_fourier_render_windows(const hh_params *p, const float *holo, int32_t nwin, int32_t hop, float *images,
                                    void *stream) {
  return fourier_windows(p, holo, nwin, hop, images, stream, "hh_fourier_render_windows");
}

hh_status hh_pipeline(const hh_params *p, const uint16_t *frames, float *image, double *evals, double *evecs,
                      int32_t *info, void *workspace, size_t ws_bytes, void *stream) {
  hh_status st;
  if ((st = check_optics(p)) || (st = check_stack(p)) || (st = check_select(p)) || (st = check_precision(p, true)))
    return st;
  if (!frames || !image) return fail(HH_E_INVALID, "frames and image must be non-NULL");
  if (!aligned(frames, frames_align(*p)) || !aligned(image, 8) || (evals && !aligned(evals, 8)) ||
      (evecs && !aligned(evecs, 16)) || (info && !aligned(info, 4)))
    return fail(HH_E_INVALID, "pipeline arrays misaligned");
  const PipeLayout L = pipe_layout(p);
  if (!workspace || ws_bytes < L.total || !aligned(workspace, 256))
    return fail(HH_E_WORKSPACE, "pipeline workspace: need %zu bytes (256-byte aligned), got %zu", L.total, ws_bytes);
  const Plan *pl = get_plan(*p);
  if (!pl) return HH_E_DEVICE;
  char *ws = static_cast<char *>(workspace);
  double *ev = evals ? evals : reinterpret_cast<double *>(ws + L.evals);
  double *V = evecs ? evecs : reinterpret_cast<double *>(ws + L.evecs);
  int *inf = info ? info : reinterpret_cast<int *>(ws + L.info);
  hipStream_t s = (hipStream_t)stream;
  StackViews v;
  hipError_t e = enqueue_front(*p, pl, L, ws, frames, nullptr, v, s);
  if (e == hipSuccess) {
    const EighProblem prob{p->nt, v.cov, ev, V, inf, v.part2, v.g2, v.D, p->eigh_solver};
    e = launch_eigh_batch(&prob, 1, 40, s);
  }
  if (e == hipSuccess) e = enqueue_back(*p, v, V, image, s);
  if (e != hipSuccess) return device_fail(e, "hh_pipeline");
  return HH_OK;
}

size_t hh_batch_workspace_bytes(const hh_params *p, int32_t n) { return batch_ws_bytes(p, n, true); }

size_t hh_analyze_batch_workspace_bytes(const hh_params *p, int32_t n) { return batch_ws_bytes(p, n, false); }

hh_status hh_pipeline_batch(const hh_params *p, int32_t n, const hh_stack *stacks, void *workspace,
                            size_t ws_bytes, void *stream) {
  if (!p || !stacks) return fail(HH_E_INVALID, "params and stacks must be non-NULL");
  if (n < 1 || n > kMaxBatch) return fail(HH_E_INVALID, "batch size n=%d must be in [1, %d]", n, kMaxBatch);
  std::vector<BatchItem> items(n);
  for (int i = 0; i < n; ++i) {
    if (!stacks[i].frames) return fail(HH_E_INVALID, "stack %d: frames must be non-NULL", i);
    if (!aligned(stacks[i].frames, 16)) return fail(HH_E_INVALID, "stack %d: frames must be 16-byte aligned", i);
    items[i] = BatchItem{stacks[i].frames, nullptr, stacks[i].image, stacks[i].evals, stacks[i].evecs, stacks[i].info};
  }
  return run_batch(p, n, items.data(), workspace, ws_bytes, (hipStream_t)stream, "hh_pipeline_batch");
}

hh_status hh_analyze_batch(const hh_params *p, int32_t n, const hh_window *wins, void *workspace, size_t ws_bytes,
                           void *stream) {
  if (!p || !wins) return fail(HH_E_INVALID, "params and windows must be non-NULL");
  if (n < 1 || n > kMaxBatch) return fail(HH_E_INVALID, "batch size n=%d must be in [1, %d]", n, kMaxBatch);
  std::vector<BatchItem> items(n);
  for (int i = 0; i < n; ++i) {
    if (!wins[i].holo) return fail(HH_E_INVALID, "window %d: holo must be non-NULL", i);
    if (!aligned(wins[i].holo, 16)) return fail(HH_E_INVALID, "window %d: holo must be 16-byte aligned", i);
    items[i] = BatchItem{nullptr, reinterpret_cast<const float2 *>(wins[i].holo), wins[i].image, wins[i].evals,
                         wins[i].evecs, wins[i].info};
  }
  return run_batch(p, n, items.data(), workspace, ws_bytes, (hipStream_t)stream, "hh_analyze_batch");
}

struct hh_graph {
  hipGraph_t graph = nullptr;
  hipGraphExec_t exec = nullptr;
  int n = 0;
};

hh_status hh_graph_create(const hh_params *p, int32_t n, const hh_stack *stacks, void *workspace, size_t ws_bytes,
                          hh_graph **out) {
  if (!out) return fail(HH_E_INVALID, "out must be non-NULL");
  *out = nullptr;
  if (!p || !stacks) return fail(HH_E_INVALID, "params and stacks must be non-NULL");
  if (n < 1 || n > kMaxBatch) return fail(HH_E_INVALID, "batch size n=%d must be in [1, %d]", n, kMaxBatch);
  std::vector<BatchItem> items(n);
  for (int i = 0; i < n; ++i) {
    if (!stacks[i].frames) return fail(HH_E_INVALID, "stack %d: frames must be non-NULL", i);
    if (!aligned(stacks[i].frames, 16)) return fail(HH_E_INVALID, "stack %d: frames must be 16-byte aligned", i);
    items[i] = BatchItem{stacks[i].frames, nullptr, stacks[i].image, stacks[i].evals, stacks[i].evecs, stacks[i].info};
    hh_status st;
    if ((st = check_optics(p + i)) || (st = check_shape(p + i))) {
      const std::string msg = g_err;
      return fail(st, "stack %d: %s", i, msg.c_str());
    }
    if (!get_plan(p[i])) return HH_E_DEVICE;  // tables allocated here, outside the capture
  }
  // the capture stream and the stream of the graph's second branch
  hipStream_t cs = nullptr, br = nullptr;
  hipError_t e = hipStreamCreateWithFlags(&cs, hipStreamNonBlocking);
  if (e == hipSuccess) e = hipStreamCreateWithFlags(&br, hipStreamNonBlocking);
  auto destroy_streams = [&]() {
    if (cs) (void)hipStreamDestroy(cs);
    if (br) (void)hipStreamDestroy(br);
  };
  if (e != hipSuccess) {
    destroy_streams();
    return device_fail(e, "hh_graph_create (stream)");
  }
  e = hipStreamBeginCapture(cs, hipStreamCaptureModeThreadLocal);
  if (e != hipSuccess) {
    destroy_streams();
    return device_fail(e, "hh_graph_create (begin capture)");
  }
  const hh_status st = run_batch(p, n, items.data(), workspace, ws_bytes, cs, "hh_graph_create", br);
  hipGraph_t graph = nullptr;
  const hipError_t e2 = hipStreamEndCapture(cs, &graph);
  destroy_streams();
  if (st != HH_OK) {
    if (graph) (void)hipGraphDestroy(graph);
    return st;
  }
  if (e2 != hipSuccess) return device_fail(e2, "hh_graph_create (end capture)");
  hipGraphExec_t exec = nullptr;
  e = hipGraphInstantiate(&exec, graph, nullptr, nullptr, 0);
  if (e != hipSuccess) {
    (void)hipGraphDestroy(graph);
    return device_fail(e, "hh_graph_create (instantiate)");
  }
  hh_graph *g = new (std::nothrow) hh_graph;
  if (!g) {
    (void)hipGraphExecDestroy(exec);
    (void)hipGraphDestroy(graph);
    return fail(HH_E_DEVICE, "hh_graph_create: out of host memory");
  }
  g->graph = graph;
  g->exec = exec;
  g->n = n;
  *out = g;
  return HH_OK;
}

hh_status hh_graph_launch(hh_graph *g, void *stream) {
  if (!g || !g->exec) return fail(HH_E_INVALID, "graph must be non-NULL");
  const hipError_t e = hipGraphLaunch(g->exec, (hipStream_t)stream);
  if (e != hipSuccess) return device_fail(e, "hh_graph_launch");
  return HH_OK;
}

void hh_graph_destroy(hh_graph *g) {
  if (!g) return;
  if (g->exec) (void)hipGraphExecDestroy(g->exec);
  if (g->graph) (void)hipGraphDestroy(g->graph);
  delete g;
}

hh_status hh_tuning_get(const hh_params *p, hh_tuning *t) {
  if (!p || !t) return fail(HH_E_INVALID, "params and tuning must be non-NULL");
  hh_status st;
  if ((st = check_shape(p))) return st;
  const Tune tu = get_tune(*p);
  *t = hh_tuning{tu.rows, tu.cols, tu.pxw, tu.group, tu.gram_ref, tu.fused};
  return HH_OK;
}

hh_status hh_tuning_set(const hh_params *p, const hh_tuning *t) {
  if (!p || !t) return fail(HH_E_INVALID, "params and tuning must be non-NULL");
  hh_status st;
  if ((st = check_shape(p)) || (st = check_tune(*p, *t))) return st;
  put_tune(*p, Tune{t->fft_rows, t->fft_cols, t->gram_pxw, t->group, t->gram_ref, t->fused});
  return HH_OK;
}

void hh_tuning_reset(void) {
  std::lock_guard<std::mutex> g(g_tune_mu);
  g_fft_tune.clear();
  g_gram_tune.clear();
}

hh_status hh_autotune(const hh_params *p, const uint16_t *frames, void *workspace, size_t ws_bytes, int32_t reps,
                      hh_tuning *best, void *stream) {
  if (!p || !frames) return fail(HH_E_INVALID, "params and frames must be non-NULL");
  if (reps < 1 || reps > 1000) return fail(HH_E_INVALID, "reps=%d must be in [1, 1000]", reps);
  hh_status st;
  if ((st = check_optics(p)) || (st = check_stack(p)) || (st = check_select(p)) || (st = check_precision(p, true)))
    return st;
  hipStream_t s = (hipStream_t)stream;
  hipStreamCaptureStatus cs = hipStreamCaptureStatusNone;
  if (hipStreamIsCapturing(s, &cs) != hipSuccess || cs != hipStreamCaptureStatusNone)
    return fail(HH_E_INVALID, "hh_autotune times real launches: not under stream capture");
  const long long npix = (long long)p->nx * p->ny;
  hipError_t e = hipSuccess;
  float *img = nullptr;
  hipEvent_t ev0 = nullptr, ev1 = nullptr;
  e = hipMalloc(&img, (size_t)npix * sizeof(float));
  if (e == hipSuccess) e = hipEventCreate(&ev0);
  if (e == hipSuccess) e = hipEventCreate(&ev1);
  // median time of `reps` pipelines under tuning t (one untimed run first)
  auto time_of = [&](const Tune &t, float &ms) -> hh_status {
    put_tune(*p, t);
    std::vector<float> v;
    for (int r = 0; r <= reps; ++r) {
      if (hipEventRecord(ev0, s) != hipSuccess) return device_fail(hipGetLastError(), "hh_autotune");
      const hh_status q = hh_pipeline(p, frames, img, nullptr, nullptr, nullptr, workspace, ws_bytes, stream);
      if (q != HH_OK) return q;
      hipError_t ee = hipEventRecord(ev1, s);
      if (ee == hipSuccess) ee = hipEventSynchronize(ev1);
      float x = 0.f;
      if (ee == hipSuccess) ee = hipEventElapsedTime(&x, ev0, ev1);
      if (ee != hipSuccess) return device_fail(ee, "hh_autotune");
      if (r > 0) v.push_back(x);
    }
    std::sort(v.begin(), v.end());
    ms = v[v.size() / 2];
    return HH_OK;
  };
  const Tune saved = get_tune(*p);
  Tune cur = saved;
  cur.rows = cur.cols = 0;
  st = e == hipSuccess ? HH_OK : device_fail(e, "hh_autotune (setup)");
  float best_ms = 0.f;
  if (st == HH_OK) st = time_of(cur, best_ms);
  // coordinate descent: row shape, column shape, group size, split-K chunk
  const int dg = default_group(*p);
  std::vector<std::pair<int Tune::*, std::vector<int>>> axes = {
      {&Tune::rows, p->nx >= 512 ? std::vector<int>{0, 1, 2, 3, 4, 5, 6, 7, 8, 9} : std::vector<int>{0}},
      {&Tune::cols, p->ny >= 512 ? std::vector<int>{0, 1, 2, 3, 4, 5, 6, 7} : std::vector<int>{0}},
      {&Tune::group, {0, std::max(1, dg / 2), std::max(1, dg / 4), std::min(2 * dg, p->nt), std::min(4 * dg, p->nt)}},
      {&Tune::pxw, {256, 512, 1024}},
      {&Tune::gram_ref, {0, 1}},
      {&Tune::fused, {1, 0}}};
  for (auto &ax : axes) {
    for (int val : ax.second) {
      if (st != HH_OK) break;
      if (cur.*(ax.first) == val) continue;
      Tune t = cur;
      t.*(ax.first) = val;
      float ms = 0.f;
      st = time_of(t, ms);
      if (st == HH_OK && ms < best_ms) {
        best_ms = ms;
        cur = t;
      }
    }
  }
  put_tune(*p, st == HH_OK ? cur : saved);
  if (img) (void)hipFree(img);
  if (ev0) (void)hipEventDestroy(ev0);
  if (ev1) (void)hipEventDestroy(ev1);
  if (st == HH_OK && best) *best = hh_tuning{cur.rows, cur.cols, cur.pxw, cur.group, cur.gram_ref, cur.fused};
  return st;
}

void hh_plan_cache_clear(void) {
  std::lock_guard<std::mutex> g(g_plan_mu);
  for (auto &kv : g_plans) {
    (void)hipFree(kv.second.chirp_x);
    (void)hipFree(kv.second.chirp_y);
    (void)hipFree(kv.second.tw_x);
    (void)hipFree(kv.second.tw_y);
  }
  g_plans.clear();
  for (auto &kv : g_dft) (void)hipFree(kv.second);
  g_dft.clear();
}

void hh_profile_enable(int32_t on) {
  std::lock_guard<std::mutex> g(g_prof_mu);
  g_prof_on = on != 0;
}

void hh_profile_reset(void) {
  std::lock_guard<std::mutex> g(g_prof_mu);
  for (auto &r : g_prof) {
    (void)hipEventSynchronize(r.b);
    g_prof_pool.push_back(r.a);
    g_prof_pool.push_back(r.b);
  }
  g_prof.clear();
}

int32_t hh_profile_read(char *buf, int32_t len) {
  std::lock_guard<std::mutex> g(g_prof_mu);
  std::map<std::string, std::pair<long long, double>> agg;
  for (auto &r : g_prof) {
    float ms = 0.f;
    if (hipEventSynchronize(r.b) == hipSuccess && hipEventElapsedTime(&ms, r.a, r.b) == hipSuccess) {
      auto &x = agg[r.name];
      x.first += 1;
      x.second += ms;
    }
  }
  std::string out = "{";
  bool first = true;
  for (auto &kv : agg) {
    char tmp[256];
    snprintf(tmp, sizeof tmp, "%s\"%s\": [%lld, %.9g]", first ? "" : ", ", kv.first.c_str(), kv.second.first,
             kv.second.second);
    out += tmp;
    first = false;
  }
  out += "}";
  if (buf && len > 0) {
    const size_t n = out.size() < (size_t)(len - 1) ? out.size() : (size_t)(len - 1);
    memcpy(buf, out.data(), n);
    buf[n] = 0;
  }
  return (int32_t)out.size() + 1;
}

}  // extern "C"
