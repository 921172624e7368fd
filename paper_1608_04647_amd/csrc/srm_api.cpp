// Host side of the SRM C-ABI: argument validation, work planning, workspace
// layout, ingestion of the data (one subject at a time, the upload of the next
// chunk overlapping the conversion of the last one), the starting maps,
// kernel sequencing, hipGraph replay of one iteration, and the snapshot that
// undoes a failed fit.  The EM arithmetic itself runs in the kernels of
// srm_kernels.hip.

#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdarg>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <string>
#include <thread>
#include <vector>

#include <sys/stat.h>

#include "../../include/srm.h"
#include "srm_internal.h"

namespace srm {
hipError_t launch_convert(hipStream_t, int, const ConvertArgs&);
hipError_t launch_rowsum(hipStream_t, int, const double*, const Subject*, double*);
hipError_t launch_seed(hipStream_t, int, const SeedArgs&);
hipError_t launch_mphase(hipStream_t, int, int, int, const MArgs&);
hipError_t launch_ephase(hipStream_t, int, int, int, const EArgs&);
hipError_t launch_ereduce(hipStream_t, int, int, int, const RArgs&);
int ereduce_ct(int kp);
int ephase_panel(int prec);  // TRs per E-phase workgroup
hipError_t launch_post_prep(hipStream_t, int, const PrepArgs&);
hipError_t launch_post_s(hipStream_t, int, int, int, const SArgs&);
hipError_t launch_post_fin(hipStream_t, int, const FinArgs&);
hipError_t launch_copy_state(hipStream_t, const CopyArgs&);
hipError_t launch_polar(hipStream_t, int, int, const QArgs&);
hipError_t launch_get_w(hipStream_t, int, const WArgs&);
hipError_t launch_transform(hipStream_t, int, int, const TArgs&, const TFArgs&);
hipError_t occupancy_mphase(int, int, int*);
hipError_t launch_map(hipStream_t, int, const MapArgs&);
hipError_t launch_gram_build(hipStream_t, int, int, int, const GBArgs&);
hipError_t launch_gram_iter(hipStream_t, int, int, const GZArgs&, const GSArgs&);
bool fused_supported(int kp, int prec, int64_t ldt);
bool fused_chunk_ok(int64_t ldt, int chunk);
hipError_t launch_fused(hipStream_t, int, int, int64_t, int, int, const FusedArgs&);
bool staged_supported(int kp, int prec, int64_t ldt);
hipError_t launch_staged(hipStream_t, int, int, int64_t, int, const FusedArgs&);
size_t static_scratch_bytes();
hipError_t static_scratch_setup(int dev);
void* static_scratch_ptr(int dev);
}  // namespace srm

using namespace srm;

namespace {

thread_local std::string g_err;

srm_status fail(srm_status s, const char* fmt, ...) {
  char buf[512];
  va_list ap;
  va_start(ap, fmt);
  vsnprintf(buf, sizeof buf, fmt, ap);
  va_end(ap);
  g_err = buf;
  return s;
}

#define HIP_OR_FAIL(expr)                                                 \
  do {                                                                    \
    hipError_t e_ = (expr);                                               \
    if (e_ != hipSuccess)                                                 \
      return fail(SRM_E_HIP, "%s failed: %s", #expr, hipGetErrorString(e_)); \
  } while (0)

int64_t round_up(int64_t x, int64_t m) { return (x + m - 1) / m * m; }

// Default launch shapes (srm_tuning; the autotuner may pick others):
//  streaming sweep workgroups: two-pass E-phase, one residency round on 256
//  CUs (two 4-wave workgroups per CU); one-pass sweep, 8-wave workgroups, two
//  equal rounds of about one per CU.  Workspace sizes cover every candidate,
//  so they do not depend on a device query.
constexpr int kSweepWGs = 512;
constexpr int kReduceWGs = 512;
constexpr int kSweepWGChoices[] = {256, 512, 768, 1024};
constexpr int kTwoPassWGChoices[] = {256, 512, 1024};
constexpr int kReduceWGChoices[] = {256, 512, 1024};
// Streamed host ingestion: each of the two device staging buffers holds up to
// this many bytes of one subject's FP32 rows.
constexpr size_t kStageBytes = (size_t)64 << 20;

struct Plan {
  int N = 0, k = 0, KP = 0, NB = 0, prec = 0;
  int64_t t = 0, ldt = 0, total_rows = 0;
  int npanel = 0, nranges = 0, nslices = 0;
  int max_nranges = 0, max_nslices = 0, max_ngrp = 0;  // over the tuning candidates
  bool fused = false;
  bool gram = false;  // sample-space iteration on G_i = Xhat_i^T Xhat_i
  int nq = 0;         // 64-TR column tiles of G_i
  int rct = 0, ncol_r = 0, gsub = 0, ngrp = 0;
  int nblk_s = 0;
  int64_t stage_rows = 0;  // rows per staging buffer (streamed host ingestion)
  std::vector<Subject> subj;
  std::vector<Slice> slices;
  std::vector<int32_t> range_slice;
  // workspace offsets (bytes)
  size_t o_xh = 0, o_xl = 0, o_mu = 0, o_isd = 0, o_rowc = 0, o_c = 0, o_arec = 0,
         o_zpart = 0, o_gpart = 0, o_p64 = 0, o_rho2 = 0, o_ygrp = 0,
         o_s64cur = 0, o_s64new = 0, o_sreccur = 0, o_srecnew = 0,
         o_sspart = 0, o_trpart = 0, o_sigcur = 0, o_signew = 0, o_M = 0,
         o_polwork = 0, o_vprev = 0, o_pjac = 0, o_sc = 0, o_ll = 0, o_subj = 0,
         o_slices = 0, o_rs = 0, o_stage = 0, o_backup = 0,
         o_G = 0, o_gz = 0, o_subjg = 0;
  size_t stage_bytes = 0;  // one staging buffer
  size_t backup_bytes = 0;
  size_t total = 0;
  size_t arec_bytes = 0, srec_bytes = 0, zpart_bytes = 0;
};

size_t esz_x(int prec) { return prec == SRM_FP32 ? 4 : 2; }

srm_status validate(const srm_desc* d) {
  if (!d) return fail(SRM_E_ARG, "desc is NULL");
  if (d->n_subjects < 1) return fail(SRM_E_ARG, "n_subjects must be >= 1");
  if (!d->v) return fail(SRM_E_ARG, "v is NULL");
  if (d->k < 1 || d->k > kMaxK)
    return fail(SRM_E_ARG, "k=%d outside [1, %d]", d->k, kMaxK);
  if (d->t < 2 || d->t > 65536)
    return fail(SRM_E_ARG, "t=%lld outside [2, 65536]", (long long)d->t);
  if (d->k > d->t) return fail(SRM_E_ARG, "k=%d exceeds t=%lld", d->k, (long long)d->t);
  if (d->prec != SRM_FP32 && d->prec != SRM_BF16 && d->prec != SRM_BF16X2)
    return fail(SRM_E_ARG, "unknown precision %d", (int)d->prec);
  for (int i = 0; i < d->n_subjects; ++i) {
    if (d->v[i] < d->k)
      return fail(SRM_E_ARG, "v[%d]=%lld is below k=%d", i, (long long)d->v[i], d->k);
    if (d->v[i] >= (int64_t)1 << 31)
      return fail(SRM_E_ARG, "v[%d]=%lld too large", i, (long long)d->v[i]);
  }
  return SRM_OK;
}

// Workspace regions carried from one iteration to the next (checkpointed,
// and snapshotted so that a failed fit can be undone).
std::vector<std::pair<size_t, size_t>> state_regions(const Plan& p);

// Equal row ranges (multiples of 32 rows) for the streaming sweep, split at
// subject ends into slices; the subjects' slice spans follow.
void layout_ranges(Plan& p, int sweep_wgs) {
  const int64_t nblk32 = p.total_rows / 32;
  p.nranges = (int)std::max<int64_t>(
      1, std::min<int64_t>(nblk32, p.fused ? sweep_wgs : sweep_wgs / p.npanel));
  p.range_slice.assign(p.nranges + 1, 0);
  p.slices.clear();
  int si = 0;
  for (int r = 0; r < p.nranges; ++r) {
    int64_t b0 = nblk32 * r / p.nranges, b1 = nblk32 * (r + 1) / p.nranges;
    p.range_slice[r] = (int32_t)p.slices.size();
    int64_t r0 = b0 * 32;
    const int64_t r1 = b1 * 32;
    while (r0 < r1) {
      while (p.subj[si].row0 + p.subj[si].vp <= r0) ++si;
      const int64_t se = std::min<int64_t>(r1, p.subj[si].row0 + p.subj[si].vp);
      Slice sl;
      sl.row0 = r0;
      sl.nrows = (int32_t)(se - r0);
      sl.subj = si;
      p.slices.push_back(sl);
      r0 = se;
    }
  }
  p.range_slice[p.nranges] = (int32_t)p.slices.size();
  p.nslices = (int)p.slices.size();
  for (auto& su : p.subj) { su.s_beg = 0; su.s_end = 0; }
  for (int s2 = p.nslices - 1; s2 >= 0; --s2) p.subj[p.slices[s2].subj].s_beg = s2;
  for (int s2 = 0; s2 < p.nslices; ++s2) p.subj[p.slices[s2].subj].s_end = s2 + 1;
}

// E-step reduction: subject groups x column tiles, about reduce_wgs in all.
void layout_reduce(Plan& p, int reduce_wgs) {
  p.ngrp = std::max(1, std::min(p.N, reduce_wgs / p.ncol_r));
  p.gsub = (p.N + p.ngrp - 1) / p.ngrp;
  p.ngrp = (p.N + p.gsub - 1) / p.gsub;
}

srm_tuning default_tuning(const Plan& p) {
  srm_tuning t{};
  // The staged one-pass kernel where it applies (measured faster at the
  // batched workload's shape), else the register-ring kernel.
  const bool staged = p.fused && staged_supported(p.KP, p.prec, p.ldt);
  t.sweep_kernel = staged ? SRM_KERNEL_STAGED : SRM_KERNEL_RING;
  t.sweep_wgs = kSweepWGs;
  t.chunk_rows = !p.fused ? 0 : staged ? 32 : (p.ldt == 512 ? 64 : (int)(16 * (p.ldt / 64)));
  t.reduce_wgs = kReduceWGs;
  t.mphase_rounds = (p.fused || p.gram) ? 0 : 1;
  return t;
}

// Every launch shape that computes this problem's sweep: the cross product of
// the sweep's own choices and the reduction's.  All compute the same EM
// iterate; they differ in the order of FP32 partial sums (so in rounding).
std::vector<srm_tuning> tuning_candidates(const Plan& p) {
  std::vector<srm_tuning> sweep;
  const srm_tuning d = default_tuning(p);
  if (p.gram) {
    sweep.push_back(d);
  } else if (p.fused) {
    for (int w : kSweepWGChoices) {
      const int own = 16 * (int)(p.ldt / 64);  // one 16-row block per wave
      std::vector<int> chunks{own};
      if (own != 64) chunks.push_back(64);
      for (int ch : chunks) {
        if (!fused_chunk_ok(p.ldt, ch)) continue;
        srm_tuning t = d;
        t.sweep_kernel = SRM_KERNEL_RING;
        t.sweep_wgs = w;
        t.chunk_rows = ch;
        sweep.push_back(t);
      }
      if (staged_supported(p.KP, p.prec, p.ldt)) {
        srm_tuning t = d;
        t.sweep_kernel = SRM_KERNEL_STAGED;
        t.sweep_wgs = w;
        t.chunk_rows = 32;
        sweep.push_back(t);
      }
    }
  } else {
    for (int w : kTwoPassWGChoices)
      for (int mr : {1, 2}) {
        srm_tuning t = d;
        t.sweep_wgs = w;
        t.mphase_rounds = mr;
        sweep.push_back(t);
      }
  }
  std::vector<srm_tuning> all;
  for (const auto& t : sweep)
    for (int r : kReduceWGChoices) {
      srm_tuning u = t;
      u.reduce_wgs = r;
      all.push_back(u);
    }
  return all;
}

bool same_tuning(const srm_tuning& a, const srm_tuning& b) {
  return a.sweep_kernel == b.sweep_kernel && a.sweep_wgs == b.sweep_wgs &&
         a.chunk_rows == b.chunk_rows && a.reduce_wgs == b.reduce_wgs &&
         a.mphase_rounds == b.mphase_rounds;
}

srm_status make_plan(const srm_desc* d, Plan& p) {
  srm_status s = validate(d);
  if (s != SRM_OK) return s;
  p.N = d->n_subjects;
  p.k = d->k;
  p.KP = (int)round_up(d->k, 16);
  p.NB = p.KP / 16;
  p.prec = d->prec;
  p.t = d->t;
  p.ldt = round_up(d->t, kColPad);
  // The one-pass sweep runs whole 128-TR groups (pairs of 64-TR waves).
  p.gram = (d->flags & SRM_GRAM) != 0;
  if (p.gram && p.N > 65535) return fail(SRM_E_ARG, "SRM_GRAM supports at most 65535 subjects");
  if (fused_supported(p.KP, p.prec, round_up(d->t, 128)) &&
      !(d->flags & (SRM_TWO_PASS | SRM_GRAM)))
    p.ldt = round_up(d->t, 128);
  p.subj.resize(p.N);
  int64_t row = 0;
  for (int i = 0; i < p.N; ++i) {
    p.subj[i].row0 = row;
    p.subj[i].v = (int32_t)d->v[i];
    p.subj[i].vp = (int32_t)round_up(d->v[i], kRowPad);
    row += p.subj[i].vp;
  }
  p.total_rows = row;
  // E-phase: equal row ranges (multiples of 32 rows) split at subject ends,
  // each swept by npanel workgroups side by side in TRs.
  p.npanel = (int)((p.ldt + ephase_panel(p.prec) - 1) / ephase_panel(p.prec));
  p.fused = fused_supported(p.KP, p.prec, p.ldt) && !(d->flags & (SRM_TWO_PASS | SRM_GRAM));
  p.rct = ereduce_ct(p.KP);
  p.ncol_r = (int)(p.ldt / p.rct);
  // Workspace for the largest range and reduction layouts of any candidate.
  for (const auto& t : tuning_candidates(p)) {
    layout_ranges(p, t.sweep_wgs);
    layout_reduce(p, t.reduce_wgs);
    p.max_nranges = std::max(p.max_nranges, p.nranges);
    p.max_nslices = std::max(p.max_nslices, p.nslices);
    p.max_ngrp = std::max(p.max_ngrp, p.ngrp);
  }
  const srm_tuning t0 = default_tuning(p);
  layout_ranges(p, t0.sweep_wgs);
  layout_reduce(p, t0.reduce_wgs);
  p.nblk_s = (int)(p.ldt / 16);

  // workspace layout
  size_t off = 0;
  auto take = [&](size_t bytes) {
    const size_t o = off;
    off = (size_t)round_up((int64_t)(off + bytes), 256);
    return o;
  };
  const size_t xplane = (size_t)p.total_rows * p.ldt * esz_x(p.prec);
  p.o_xh = take(xplane);
  p.o_xl = p.prec == SRM_BF16X2 ? take(xplane) : p.o_xh;
  p.o_mu = take(sizeof(double) * p.total_rows);
  p.o_isd = take(sizeof(double) * p.total_rows);
  p.o_rowc = take(sizeof(double) * p.total_rows);
  p.o_c = take(sizeof(double) * p.N);
  p.arec_bytes = (size_t)p.total_rows * p.KP * 4;  // FP32, or 2 bf16 planes
  p.o_arec = take(p.arec_bytes);
  p.zpart_bytes = (size_t)p.max_nslices * p.KP * p.ldt * 4;
  p.o_zpart = take(p.zpart_bytes);
  p.o_gpart = take((size_t)p.max_nslices * p.KP * p.KP * 4);
  p.o_p64 = take((size_t)p.N * p.KP * p.KP * 8);
  p.o_rho2 = take(sizeof(double) * p.N);
  p.o_ygrp = take((size_t)p.max_ngrp * p.KP * p.ldt * 8);
  p.o_s64cur = take((size_t)p.KP * p.ldt * 8);
  p.o_s64new = take((size_t)p.KP * p.ldt * 8);
  p.srec_bytes = (size_t)p.KP * p.ldt * 4;
  p.o_sreccur = take(p.srec_bytes);
  p.o_srecnew = take(p.srec_bytes);
  p.o_sspart = take((size_t)p.nblk_s * p.KP * p.KP * 8);
  p.o_trpart = take((size_t)p.nblk_s * 8);
  p.o_sigcur = take((size_t)p.KP * p.KP * 8);
  p.o_signew = take((size_t)p.KP * p.KP * 8);
  p.o_M = take((size_t)p.KP * p.KP * 8);
  p.o_polwork = take(p.KP > 80 ? (size_t)p.N * 3 * p.KP * (p.KP + 1) * 8 : 8);
  p.o_vprev = take((size_t)p.N * p.KP * p.KP * 8);
  p.o_pjac = take(sizeof(int32_t) * p.N);
  p.o_sc = take(sizeof(Scalars));
  p.o_ll = take(sizeof(double) * kLLCapacity);
  p.o_subj = take(sizeof(Subject) * p.N);
  p.o_slices = take(sizeof(Slice) * p.max_nslices);
  p.o_rs = take(sizeof(int32_t) * (p.max_nranges + 1));
  if (p.gram) {
    p.nq = (int)(p.ldt / 64);
    if ((int64_t)p.nq * (p.nq + 1) / 2 * p.N >= ((int64_t)1 << 31))
      return fail(SRM_E_ARG, "SRM_GRAM: too many Gram tiles (t or N too large)");
    // FP32 storage keeps G_i in FP64 (and runs its products in FP64).
    p.o_G = take((size_t)p.N * p.ldt * p.ldt * (p.prec == SRM_FP32 ? 8 : 4));
    p.o_gz = take((size_t)p.N * p.nq * p.KP * p.KP * 8);
    p.o_subjg = take(sizeof(Subject) * p.N);
  }
  if (d->flags & SRM_X_HOST) {  // two staging buffers for FP32 rows of one subject
    int64_t vmax = 0;
    for (int i = 0; i < p.N; ++i) vmax = std::max<int64_t>(vmax, d->v[i]);
    const int64_t row_bytes = p.t * (int64_t)sizeof(float);
    p.stage_rows = std::max<int64_t>(1, std::min<int64_t>(vmax, (int64_t)kStageBytes / row_bytes));
    p.stage_bytes = (size_t)(p.stage_rows * row_bytes);
    p.o_stage = take(2 * p.stage_bytes);
  }
  p.backup_bytes = 0;
  for (const auto& r : state_regions(p)) p.backup_bytes += r.second;
  p.o_backup = take(p.backup_bytes);
  p.total = off;
  return SRM_OK;
}

std::vector<std::pair<size_t, size_t>> state_regions(const Plan& p) {
  const size_t kk = (size_t)p.KP * p.KP * 8;
  return {{p.o_s64cur, (size_t)p.KP * p.ldt * 8}, {p.o_s64new, (size_t)p.KP * p.ldt * 8},
          {p.o_sreccur, p.srec_bytes},            {p.o_srecnew, p.srec_bytes},
          {p.o_sigcur, kk},                       {p.o_signew, kk},
          {p.o_M, kk},                            {p.o_rho2, sizeof(double) * p.N},
          {p.o_p64, (size_t)p.N * kk},            {p.o_vprev, (size_t)p.N * kk},
          {p.o_sc, sizeof(Scalars)},              {p.o_ll, sizeof(double) * kLLCapacity}};
}

}  // namespace

struct srm_ctx {
  Plan p;
  uint32_t flags = 0;
  uint64_t seed = 0;
  int device = 0;                 // current device at srm_init_begin
  hipError_t scratch_err = hipSuccess;  // set-up of the static scratch on it
  hipStream_t stream = nullptr;   // every kernel
  hipStream_t cstream = nullptr;  // uploads of streamed host ingestion
  bool own_stream = false;
  hipEvent_t ev_up[2] = {};       // staging buffer b filled (copy stream)
  hipEvent_t ev_conv[2] = {};     // staging buffer b converted (compute stream)
  int64_t stage_seq = 0;          // staging buffers used so far
  char* ws = nullptr;
  int m_grid = 0, m_occ = 1, m_ncu = 256;
  int64_t m_tpw = 0, m_ntiles = 0;
  int iters = 0;
  bool ready = false;             // srm_init_end completed
  bool w0_checked = false;        // srm_init checked every W0_i before ingesting
  std::vector<char> ingested;     // per subject, between init_begin and init_end
  std::vector<char> seeded;       // per subject: start drawn by the library
  srm_tuning tune{};               // launch shapes in use
  bool graph_ok = false;
  bool capture_failed = false;    // capture or instantiation failed once
  bool graph_used = false;        // the last srm_fit replayed the captured graph
  bool a_valid = true;            // A records in HBM match the current S (two-pass)
  hipGraph_t graph = nullptr;
  hipGraphExec_t gexec = nullptr;
  // Per-kernel HIP events for srm_profile (direct launches only).
  bool profiling = false;
  bool recorded[SRM_NPHASE] = {};
  hipEvent_t ev[2 * SRM_NPHASE] = {};

  template <class T>
  T* at(size_t off) const { return reinterpret_cast<T*>(ws + off); }
};

namespace {

// A-record index of element (global row R, feature b).
inline size_t arec_index(int NB, int64_t R, int b) {
  const int64_t rb = R >> 5;
  const int rr = (int)(R & 31);
  const int g = (rr & 15) >> 2, e = ((rr >> 4) << 2) + (rr & 3);
  const int lane = (b & 15) + 16 * g;
  return (size_t)(((rb * NB + (b >> 4)) * 64 + lane) * 8 + e);
}

inline uint16_t host_f2bf(float f) {
  uint32_t u;
  std::memcpy(&u, &f, 4);
  u += 0x7fffu + ((u >> 16) & 1u);
  return (uint16_t)(u >> 16);
}
inline float host_bf2f(uint16_t h) {
  uint32_t u = (uint32_t)h << 16;
  float f;
  std::memcpy(&f, &u, 4);
  return f;
}

int n_threads() {
  unsigned n = std::thread::hardware_concurrency();
  return (int)std::max(1u, std::min(16u, n ? n : 1u));
}

template <class F>
void parallel_for(int n, F f) {
  const int nt = std::min(n, n_threads());
  std::vector<std::thread> th;
  for (int w = 0; w < nt; ++w)
    th.emplace_back([&, w] { for (int i = w; i < n; i += nt) f(i); });
  for (auto& x : th) x.join();
}

// max |W0^T W0 - I| of one subject's v x k map, over row blocks in parallel.
double w0_error(const double* w, int v, int k) {
  const int nt = std::max(1, std::min(n_threads(), v / 4096 + 1));
  std::vector<std::vector<double>> part(nt, std::vector<double>((size_t)k * k, 0.0));
  parallel_for(nt, [&](int t) {
    double* g = part[t].data();
    for (int r = (int)((int64_t)v * t / nt); r < (int)((int64_t)v * (t + 1) / nt); ++r) {
      const double* row = w + (size_t)r * k;
      for (int a = 0; a < k; ++a) {
        const double x = row[a];
        double* ga = g + (size_t)a * k;
        for (int b = a; b < k; ++b) ga[b] += x * row[b];
      }
    }
  });
  double m = 0.0;
  for (int a = 0; a < k; ++a)
    for (int b = a; b < k; ++b) {
      double s = 0.0;
      for (int t = 0; t < nt; ++t) s += part[t][(size_t)a * k + b];
      m = std::max(m, std::fabs(s - (a == b ? 1.0 : 0.0)));
    }
  return m;
}

// W0_i -> subject i's A records (A = W0, deferred polar factor P = I).
srm_status upload_w0(srm_ctx* c, int i, const double* W0) {
  const Plan& p = c->p;
  const Subject& su = p.subj[i];
  const size_t nrec_el = (size_t)su.vp * p.KP;  // elements in its records
  const size_t base = arec_index(p.NB, su.row0, 0);
  std::vector<char> buf(nrec_el * 4, 0);
  const int nt = std::max(1, std::min(n_threads(), su.v / 4096 + 1));
  if (p.prec == SRM_FP32) {
    float* f = reinterpret_cast<float*>(buf.data());
    parallel_for(nt, [&](int t) {
      for (int r = (int)((int64_t)su.v * t / nt); r < (int)((int64_t)su.v * (t + 1) / nt); ++r)
        for (int b = 0; b < p.k; ++b)
          f[arec_index(p.NB, su.row0 + r, b) - base] = (float)W0[(size_t)r * p.k + b];
    });
    HIP_OR_FAIL(hipMemcpyAsync(c->ws + p.o_arec + base * 4, buf.data(), nrec_el * 4,
                               hipMemcpyHostToDevice, c->stream));
  } else {
    uint16_t* hi = reinterpret_cast<uint16_t*>(buf.data());
    uint16_t* lo = hi + nrec_el;
    parallel_for(nt, [&](int t) {
      for (int r = (int)((int64_t)su.v * t / nt); r < (int)((int64_t)su.v * (t + 1) / nt); ++r)
        for (int b = 0; b < p.k; ++b) {
          const float f = (float)W0[(size_t)r * p.k + b];
          const uint16_t h = host_f2bf(f);
          const size_t o = arec_index(p.NB, su.row0 + r, b) - base;
          hi[o] = h;
          lo[o] = host_f2bf(f - host_bf2f(h));
        }
    });
    const size_t plane = p.arec_bytes / 2;
    HIP_OR_FAIL(hipMemcpyAsync(c->ws + p.o_arec + base * 2, hi, nrec_el * 2,
                               hipMemcpyHostToDevice, c->stream));
    HIP_OR_FAIL(hipMemcpyAsync(c->ws + p.o_arec + plane + base * 2, lo, nrec_el * 2,
                               hipMemcpyHostToDevice, c->stream));
  }
  // buf is released on return: the copies must have read it.
  HIP_OR_FAIL(hipStreamSynchronize(c->stream));
  return SRM_OK;
}

struct Ptrs {
  void *xh, *xl, *ah, *al, *shc, *slc, *shn, *sln;
};

// Brackets one kernel of phase ph with HIP events when profiling.
struct Phase {
  srm_ctx* c;
  int ph;
  Phase(srm_ctx* cc, int p) : c(cc), ph(p) {
    if (c->profiling) {
      (void)hipEventRecord(c->ev[2 * ph], c->stream);
      c->recorded[ph] = true;
    }
  }
  ~Phase() {
    if (c->profiling) (void)hipEventRecord(c->ev[2 * ph + 1], c->stream);
  }
};

Ptrs ptrs(const srm_ctx* c) {
  const Plan& p = c->p;
  Ptrs q;
  q.xh = c->ws + p.o_xh;
  q.xl = c->ws + p.o_xl;
  q.ah = c->ws + p.o_arec;
  q.al = c->ws + p.o_arec + (p.prec == SRM_FP32 ? 0 : p.arec_bytes / 2);
  q.shc = c->ws + p.o_sreccur;
  q.slc = c->ws + p.o_sreccur + p.srec_bytes / 2;
  q.shn = c->ws + p.o_srecnew;
  q.sln = c->ws + p.o_srecnew + p.srec_bytes / 2;
  return q;
}

// E-phase + reduction + posterior: from the current A, P, rho produce the
// E-step's S (into the "new" buffers), Sigma_s_new, tau_new and one LL.
//  with_polar: the polar step of an iteration (P_i and rho_i^2 from G_i);
//  init_polar: the first E-step of a drawn start (P_i = (A_i^T A_i)^-1/2 of
//              the Gaussian in the A records; rho_i^2 stays 1);
//  stream_pass: the E-phase partials come from a pass over Xhat (else the
//              sample-space products have written them).
hipError_t enqueue_estep(srm_ctx* c, bool with_polar, bool stream_pass, bool init_polar) {
  const Plan& p = c->p;
  const Ptrs q = ptrs(c);
  hipStream_t st = c->stream;
  hipError_t e;
  const Scalars* sc = c->at<Scalars>(p.o_sc);
  const bool polar = with_polar || init_polar;
  EArgs ea{q.xh, q.xl, q.ah, q.al, c->at<Slice>(p.o_slices),
           c->at<int32_t>(p.o_rs), c->at<float>(p.o_zpart), c->at<float>(p.o_gpart),
           p.ldt, p.npanel, polar ? 1 : 0, sc};
  if (stream_pass) {
    Phase ph(c, SRM_PHASE_EPHASE);
    if ((e = launch_ephase(st, p.KP, p.prec, p.nranges * p.npanel, ea)) != hipSuccess) return e;
  }
  // The sample-space iteration keeps each subject's partials in slice i.
  const size_t o_tab = (p.gram && !stream_pass) ? p.o_subjg : p.o_subj;
  if (polar) {
    QArgs qa{c->at<float>(p.o_gpart), c->at<Subject>(o_tab), c->at<double>(p.o_c),
             c->at<double>(p.o_rho2), c->at<double>(p.o_p64), c->at<double>(p.o_polwork),
             c->at<double>(p.o_vprev), c->at<int32_t>(p.o_pjac), c->at<Scalars>(p.o_sc),
             p.k, p.t, init_polar ? 1 : 0};
    Phase ph(c, SRM_PHASE_POLAR);
    if ((e = launch_polar(st, p.KP, p.N, qa)) != hipSuccess) return e;
  }
  RArgs ra{c->at<float>(p.o_zpart), c->at<Subject>(o_tab), c->at<double>(p.o_p64),
           c->at<double>(p.o_rho2), c->at<double>(p.o_ygrp), p.N, p.gsub, p.ldt, sc};
  {
    Phase ph(c, SRM_PHASE_EREDUCE);
    if ((e = launch_ereduce(st, p.KP, p.ncol_r, p.ngrp, ra)) != hipSuccess) return e;
  }
  PrepArgs pa{c->at<double>(p.o_rho2), c->at<double>(p.o_c), c->at<Subject>(p.o_subj),
              c->at<double>(p.o_sigcur), c->at<double>(p.o_M),
              c->at<Scalars>(p.o_sc), p.N, p.k};
  Phase ph(c, SRM_PHASE_POSTERIOR);
  if ((e = launch_post_prep(st, p.KP, pa)) != hipSuccess) return e;
  SArgs sa{c->at<double>(p.o_ygrp), c->at<double>(p.o_M), c->at<double>(p.o_s64new),
           q.shn, q.sln, c->at<double>(p.o_sspart), c->at<double>(p.o_trpart),
           p.ngrp, p.k, p.t, p.ldt, sc};
  if ((e = launch_post_s(st, p.KP, p.prec, p.nblk_s, sa)) != hipSuccess) return e;
  double Vtot = 0.0;
  for (const auto& su : p.subj) Vtot += su.v;
  FinArgs fa{c->at<double>(p.o_sspart), c->at<double>(p.o_trpart), c->at<double>(p.o_M),
             c->at<double>(p.o_signew), c->at<double>(p.o_ll), c->at<Scalars>(p.o_sc),
             p.nblk_s, p.k, p.t, Vtot};
  return launch_post_fin(st, p.KP, fa);
}

// One EM iteration: M-step on the current posterior, then the next E-step.
hipError_t enqueue_iteration(srm_ctx* c) {
  const Plan& p = c->p;
  const Ptrs q = ptrs(c);
  hipStream_t st = c->stream;
  hipError_t e;
  const Scalars* sc = c->at<Scalars>(p.o_sc);
  CopyArgs ca{c->at<double>(p.o_s64new), c->at<double>(p.o_s64cur),
              c->at<uint4>(p.o_srecnew), c->at<uint4>(p.o_sreccur),
              c->at<double>(p.o_signew), c->at<double>(p.o_sigcur), c->at<Scalars>(p.o_sc),
              (int64_t)p.KP * p.ldt, (int64_t)(p.srec_bytes / 16), p.KP * p.KP};
  if ((e = launch_copy_state(st, ca)) != hipSuccess) return e;
  if (p.gram) {
    const bool g64 = p.prec == SRM_FP32;
    GZArgs za{g64 ? nullptr : c->at<float>(p.o_G), g64 ? c->at<double>(p.o_G) : nullptr,
              c->at<double>(p.o_s64cur), c->at<float>(p.o_zpart),
              c->at<double>(p.o_gz), p.t, p.ldt, p.nq, p.k, sc};
    GSArgs ga{c->at<double>(p.o_gz), c->at<float>(p.o_gpart), p.nq, sc};
    {
      Phase ph(c, SRM_PHASE_GRAM);
      if ((e = launch_gram_iter(st, p.KP, p.N, za, ga)) != hipSuccess) return e;
    }
    c->a_valid = false;
    return enqueue_estep(c, true, /*stream_pass=*/false, false);
  }
  if (p.fused) {
    FusedArgs fa{q.xh, q.xl, q.shc, q.slc, c->at<Slice>(p.o_slices), c->at<int32_t>(p.o_rs),
                 c->at<float>(p.o_zpart), c->at<float>(p.o_gpart), p.ldt, sc};
    {
      Phase ph(c, SRM_PHASE_FUSED);
      e = c->tune.sweep_kernel == SRM_KERNEL_STAGED
              ? launch_staged(st, p.KP, p.prec, p.ldt, p.nranges, fa)
              : launch_fused(st, p.KP, p.prec, p.ldt, p.nranges, c->tune.chunk_rows, fa);
      if (e != hipSuccess) return e;
    }
    c->a_valid = false;
    return enqueue_estep(c, true, /*stream_pass=*/false, false);
  }
  MArgs ma{q.xh, q.xl, q.shc, q.slc, q.ah, q.al, p.ldt, 0, p.total_rows, c->m_ntiles, c->m_tpw,
           sc};
  {
    Phase ph(c, SRM_PHASE_MPHASE);
    if ((e = launch_mphase(st, p.KP, p.prec, c->m_grid, ma)) != hipSuccess) return e;
  }
  c->a_valid = true;
  return enqueue_estep(c, true, /*stream_pass=*/true, false);
}

srm_status run_iterations(srm_ctx* c, int n) {
  c->graph_used = false;
  for (int it = 0; it < n; ++it) {
    if (!(c->flags & SRM_NO_GRAPH) && !c->capture_failed && !c->graph_ok) {
      // Capture one iteration once; if capture or instantiation fails the
      // iterations are launched directly (srm_get_info reports which ran).
      hipError_t e = hipStreamBeginCapture(c->stream, hipStreamCaptureModeThreadLocal);
      if (e == hipSuccess) {
        hipError_t e2 = enqueue_iteration(c);
        hipGraph_t g = nullptr;
        hipError_t e3 = hipStreamEndCapture(c->stream, &g);
        if (e2 == hipSuccess && e3 == hipSuccess && g) {
          if (hipGraphInstantiate(&c->gexec, g, nullptr, nullptr, 0) == hipSuccess) {
            c->graph = g;
            c->graph_ok = true;
          } else {
            (void)hipGraphDestroy(g);
            c->gexec = nullptr;
          }
        } else if (g) {
          (void)hipGraphDestroy(g);
        }
      }
      (void)hipGetLastError();
      if (!c->graph_ok) c->capture_failed = true;
    }
    if (c->graph_ok) {
      HIP_OR_FAIL(hipGraphLaunch(c->gexec, c->stream));
      c->graph_used = true;
    } else {
      HIP_OR_FAIL(enqueue_iteration(c));
    }
    ++c->iters;
  }
  return SRM_OK;
}

srm_status read_scalars(srm_ctx* c, Scalars* s) {
  HIP_OR_FAIL(hipMemcpyAsync(s, c->ws + c->p.o_sc, sizeof(Scalars),
                             hipMemcpyDeviceToHost, c->stream));
  HIP_OR_FAIL(hipStreamSynchronize(c->stream));
  if (s->status == SRM_E_RANK)
    return fail(SRM_E_RANK, "A_i^T A_i is numerically singular for some subject");
  if (s->status == SRM_E_NOTPD)
    return fail(SRM_E_NOTPD, "Sigma_s or Sigma_s^-1 + rho0 I is not positive definite");
  if (s->status != 0) return fail((srm_status)s->status, "device error %d", s->status);
  return SRM_OK;
}

// Copies the carried state into the backup region (save) or back (restore).
hipError_t copy_state_regions(srm_ctx* c, bool save) {
  const Plan& p = c->p;
  size_t pos = p.o_backup;
  for (const auto& r : state_regions(p)) {
    char* live = c->ws + r.first;
    char* bak = c->ws + pos;
    const hipError_t e = hipMemcpyAsync(save ? bak : live, save ? live : bak, r.second,
                                        hipMemcpyDeviceToDevice, c->stream);
    if (e != hipSuccess) return e;
    pos += r.second;
  }
  return hipSuccess;
}

// After a numeric failure inside srm_fit / srm_profile: the carried state
// goes back to what it was when the call started (the failing iteration and
// those after it returned at once on the raised status).
srm_status undo_failed_call(srm_ctx* c, int first_iter, srm_status err) {
  const std::string msg = g_err;
  if (copy_state_regions(c, false) != hipSuccess || hipStreamSynchronize(c->stream) != hipSuccess)
    return fail(SRM_E_HIP, "%s; restoring the state failed", msg.c_str());
  c->iters = first_iter;
  c->a_valid = false;
  g_err = msg;
  return err;
}

// Puts launch shape t (one of tuning_candidates) in place: the range and
// reduction layouts, their device tables, the M-phase grid; the captured
// graph (whose launches carried the old shapes) is dropped.
srm_status apply_tuning(srm_ctx* c, const srm_tuning& t) {
  Plan& P = c->p;
  bool ok = false;
  for (const auto& u : tuning_candidates(P)) ok = ok || same_tuning(u, t);
  if (!ok)
    return fail(SRM_E_ARG, "launch shape (kernel %d, %d sweep workgroups, chunk %d, %d reduce "
                "workgroups, %d M-phase rounds) is not a candidate for this problem",
                t.sweep_kernel, t.sweep_wgs, t.chunk_rows, t.reduce_wgs, t.mphase_rounds);
  layout_ranges(P, t.sweep_wgs);
  layout_reduce(P, t.reduce_wgs);
  auto up = [&](size_t off, const void* src, size_t n) {
    return hipMemcpyAsync(c->ws + off, src, n, hipMemcpyHostToDevice, c->stream);
  };
  HIP_OR_FAIL(up(P.o_subj, P.subj.data(), sizeof(Subject) * P.N));
  HIP_OR_FAIL(up(P.o_slices, P.slices.data(), sizeof(Slice) * P.nslices));
  HIP_OR_FAIL(up(P.o_rs, P.range_slice.data(), sizeof(int32_t) * (P.nranges + 1)));
  HIP_OR_FAIL(hipStreamSynchronize(c->stream));  // the host tables are rebuilt later
  // M-phase grid: mphase_rounds residency rounds of equal contiguous tile ranges.
  c->m_ntiles = (P.total_rows + 63) / 64;
  const int64_t want = (int64_t)c->m_occ * c->m_ncu * std::max(1, t.mphase_rounds);
  c->m_tpw = std::max<int64_t>(1, (c->m_ntiles + want - 1) / want);
  c->m_grid = (int)((c->m_ntiles + c->m_tpw - 1) / c->m_tpw);
  c->tune = t;
  if (c->gexec) (void)hipGraphExecDestroy(c->gexec);
  if (c->graph) (void)hipGraphDestroy(c->graph);
  c->gexec = nullptr;
  c->graph = nullptr;
  c->graph_ok = false;
  return SRM_OK;
}

srm_status check_ready(const srm_ctx* c) {
  if (!c) return fail(SRM_E_ARG, "ctx is NULL");
  if (!c->ready) return fail(SRM_E_STATE, "srm_init_end has not completed");
  return SRM_OK;
}

// Milliseconds per iteration of launch shape t: one warm-up iteration and
// `trials` timed ones (direct launches, HIP events on the context's stream),
// after which the carried state is put back as it was.  *bad receives the
// status an iteration raised (0: none).
// Times `trials` iterations of shape t after one warm-up: the phases the
// shapes change (M-phase, E-phase, one-pass sweep, sample-space products,
// E-step reduction), each bracketed by HIP events as in srm_profile; the polar
// and posterior steps are left out, since their time does not depend on the
// shapes and varies from one iteration to the next (cold and warm polar
// solves).
srm_status time_tuning(srm_ctx* c, const srm_tuning& t, int trials, double* ms, int* bad) {
  srm_status st = apply_tuning(c, t);
  if (st != SRM_OK) return st;
  for (int i = 0; i < 2 * SRM_NPHASE; ++i)
    if (!c->ev[i]) HIP_OR_FAIL(hipEventCreate(&c->ev[i]));
  HIP_OR_FAIL(enqueue_iteration(c));
  double sum = 0.0;
  for (int i = 0; i < trials; ++i) {
    for (auto& r : c->recorded) r = false;
    c->profiling = true;
    const hipError_t e = enqueue_iteration(c);
    c->profiling = false;
    HIP_OR_FAIL(e);
    HIP_OR_FAIL(hipStreamSynchronize(c->stream));
    // The posterior reads one partial of the reduction per subject group, so
    // the reduction's shape changes its time as well.
    for (int ph : {SRM_PHASE_MPHASE, SRM_PHASE_EPHASE, SRM_PHASE_FUSED, SRM_PHASE_GRAM,
                   SRM_PHASE_EREDUCE, SRM_PHASE_POSTERIOR}) {
      if (!c->recorded[ph]) continue;
      float f = 0.f;
      HIP_OR_FAIL(hipEventElapsedTime(&f, c->ev[2 * ph], c->ev[2 * ph + 1]));
      sum += f;
    }
  }
  *ms = sum / trials;
  Scalars sc{};
  HIP_OR_FAIL(hipMemcpyAsync(&sc, c->ws + c->p.o_sc, sizeof sc, hipMemcpyDeviceToHost,
                             c->stream));
  HIP_OR_FAIL(copy_state_regions(c, false));
  HIP_OR_FAIL(hipStreamSynchronize(c->stream));
  *bad = sc.status;
  return SRM_OK;
}

// On-disk cache of tuned shapes: one line per problem, "key<TAB>kernel
// sweep_wgs chunk reduce_wgs mphase_rounds<TAB>ms"; the last line of a key
// wins.  The file is $SRM_TUNE_CACHE (empty: no cache), else
// $HOME/.cache/srm_tune.tsv.
std::string tune_cache_path() {
  const char* e = std::getenv("SRM_TUNE_CACHE");
  if (e) return std::string(e);
  const char* h = std::getenv("HOME");
  if (!h || !*h) return std::string();
  return std::string(h) + "/.cache/srm_tune.tsv";
}

std::string tune_key(const srm_ctx* c) {
  const Plan& p = c->p;
  hipDeviceProp_t prop{};
  std::string arch = "unknown";
  int ncu = 0;
  if (hipGetDeviceProperties(&prop, c->device) == hipSuccess) {
    arch = prop.gcnArchName;
    ncu = prop.multiProcessorCount;
  }
  for (auto& ch : arch)
    if (ch == '\t' || ch == ' ' || ch == '\n') ch = '_';
  char buf[256];
  // "trial=2": trials time the posterior too; entries timed without it are
  // not reused.
  snprintf(buf, sizeof buf, "trial=2 %s/%dcu prec=%d kp=%d ldt=%lld sweep=%d n=%d rows=%lld",
           arch.c_str(), ncu, p.prec, p.KP, (long long)p.ldt,
           p.gram ? 2 : (p.fused ? 0 : 1), p.N, (long long)p.total_rows);
  return std::string(buf);
}

bool tune_cache_find(const srm_ctx* c, srm_tuning* t) {
  const std::string path = tune_cache_path();
  if (path.empty()) return false;
  FILE* f = std::fopen(path.c_str(), "r");
  if (!f) return false;
  const std::string key = tune_key(c);
  char line[512];
  bool found = false;
  while (std::fgets(line, sizeof line, f)) {
    const char* tab = std::strchr(line, '\t');
    if (!tab || (size_t)(tab - line) != key.size() || std::strncmp(line, key.c_str(), key.size()))
      continue;
    srm_tuning u{};
    if (std::sscanf(tab + 1, "%d %d %d %d %d", &u.sweep_kernel, &u.sweep_wgs, &u.chunk_rows,
                    &u.reduce_wgs, &u.mphase_rounds) == 5) {
      *t = u;
      found = true;
    }
  }
  std::fclose(f);
  return found;
}

void tune_cache_store(const srm_ctx* c, const srm_tuning& t, double ms) {
  const std::string path = tune_cache_path();
  if (path.empty()) return;
  const size_t slash = path.rfind('/');
  if (slash != std::string::npos && slash > 0) (void)mkdir(path.substr(0, slash).c_str(), 0755);
  FILE* f = std::fopen(path.c_str(), "a");
  if (!f) return;
  std::fprintf(f, "%s\t%d %d %d %d %d\t%.4f\n", tune_key(c).c_str(), t.sweep_kernel,
               t.sweep_wgs, t.chunk_rows, t.reduce_wgs, t.mphase_rounds, ms);
  std::fclose(f);
}

}  // namespace

// ---- checkpoint -----------------------------------------------------------

namespace {

struct StateHeader {
  char magic[8];
  uint32_t version;
  int32_t N, k, KP, prec;
  int32_t fused, iters;
  int64_t t, ldt, total_rows;
  uint64_t vhash;
  uint64_t bytes;
};

constexpr char kStateMagic[8] = {'S', 'R', 'M', 'S', 'T', 'A', 'T', 'E'};
constexpr uint32_t kStateVersion = 2;

uint64_t hash_v(const Plan& p) {  // FNV-1a over the voxel counts
  uint64_t h = 1469598103934665603ull;
  for (const auto& su : p.subj) {
    uint64_t x = (uint64_t)su.v;
    for (int b = 0; b < 8; ++b) {
      h ^= (x >> (8 * b)) & 0xff;
      h *= 1099511628211ull;
    }
  }
  return h;
}

size_t state_bytes(const Plan& p) {
  size_t n = sizeof(StateHeader) + sizeof(double) * p.N;  // header, c_i
  for (const auto& r : state_regions(p)) n += r.second;
  return n;
}

StateHeader make_header(const srm_ctx* c) {
  const Plan& p = c->p;
  StateHeader h{};
  std::memcpy(h.magic, kStateMagic, 8);
  h.version = kStateVersion;
  h.N = p.N;
  h.k = p.k;
  h.KP = p.KP;
  h.prec = p.prec;
  h.fused = p.fused ? 1 : (p.gram ? 2 : 0);
  h.iters = c->iters;
  h.t = p.t;
  h.ldt = p.ldt;
  h.total_rows = p.total_rows;
  h.vhash = hash_v(p);
  h.bytes = state_bytes(p);
  return h;
}

// Conversion of subject i's FP32 rows [r0, r0 + n) (subject-local) from src.
hipError_t convert_rows(srm_ctx* c, int i, const float* src, int64_t r0, int64_t n, bool last) {
  const Plan& P = c->p;
  const Ptrs q = ptrs(c);
  const Subject& su = P.subj[i];
  // The chunk that ends the subject also converts its zero padding rows.
  const int64_t row_begin = su.row0 + r0;
  const int64_t row_end = last ? su.row0 + su.vp : su.row0 + r0 + n;
  ConvertArgs ca{src, r0, su.row0, su.v, P.t, P.ldt, row_begin, row_end, q.xh, q.xl,
                 c->at<double>(P.o_mu), c->at<double>(P.o_isd), c->at<double>(P.o_rowc),
                 c->at<Scalars>(P.o_sc), P.prec, (c->flags & SRM_ZSCORE) ? 1 : 0};
  return launch_convert(c->stream, (int)((row_end - row_begin + 3) / 4), ca);
}

}  // namespace

extern "C" {

srm_status srm_workspace_size(const srm_desc* desc, size_t* bytes) {
  if (!bytes) return fail(SRM_E_ARG, "bytes is NULL");
  Plan p;
  srm_status s = make_plan(desc, p);
  if (s != SRM_OK) return s;
  *bytes = p.total;
  return SRM_OK;
}

srm_status srm_init_begin(srm_ctx** out, const srm_desc* desc, uint64_t seed, void* workspace,
                          size_t ws_bytes) {
  if (!out) return fail(SRM_E_ARG, "out is NULL");
  *out = nullptr;
  Plan p;
  srm_status s = make_plan(desc, p);
  if (s != SRM_OK) return s;
  if (!workspace) return fail(SRM_E_WORKSPACE, "workspace is NULL");
  if (((uintptr_t)workspace & 255) != 0)
    return fail(SRM_E_WORKSPACE, "workspace must be 256-byte aligned");
  if (ws_bytes < p.total)
    return fail(SRM_E_WORKSPACE, "workspace has %zu bytes, %zu needed", ws_bytes, p.total);

  srm_ctx* c = new srm_ctx();
  c->p = std::move(p);
  c->flags = desc->flags;
  c->seed = seed;
  c->ws = static_cast<char*>(workspace);
  const Plan& P = c->p;
  c->ingested.assign(P.N, 0);
  c->seeded.assign(P.N, 0);
  if (desc->hip_stream) {
    c->stream = static_cast<hipStream_t>(desc->hip_stream);
  } else {
    if (hipStreamCreateWithFlags(&c->stream, hipStreamNonBlocking) != hipSuccess) {
      delete c;
      return fail(SRM_E_HIP, "hipStreamCreateWithFlags failed");
    }
    c->own_stream = true;
  }
  auto bail = [&](srm_status st) {
    const std::string msg = g_err;
    srm_free(c);
    g_err = msg;
    return st;
  };
  if (c->flags & SRM_X_HOST) {
    // Uploads run on a second stream (same default priority), so that the
    // conversion of one staging buffer overlaps the upload of the other.
    if (hipStreamCreateWithFlags(&c->cstream, hipStreamNonBlocking) != hipSuccess)
      return bail(fail(SRM_E_HIP, "hipStreamCreateWithFlags failed"));
    for (int b = 0; b < 2; ++b)
      if (hipEventCreateWithFlags(&c->ev_up[b], hipEventDisableTiming) != hipSuccess ||
          hipEventCreateWithFlags(&c->ev_conv[b], hipEventDisableTiming) != hipSuccess)
        return bail(fail(SRM_E_HIP, "hipEventCreate failed"));
  }

  // The static scratch of srm_transform_static: its address on this device
  // (looked up once per device; a failure only disables that entry point).
  if (hipGetDevice(&c->device) != hipSuccess) c->device = 0;
  c->scratch_err = static_scratch_setup(c->device);

  // M-phase occupancy, for its grid (apply_tuning).
  int occ = 0;
  if (occupancy_mphase(P.KP, P.prec, &occ) != hipSuccess || occ < 1) occ = 1;
  int dev = 0, ncu = 256;
  if (hipGetDevice(&dev) == hipSuccess) {
    hipDeviceProp_t prop;
    if (hipGetDeviceProperties(&prop, dev) == hipSuccess && prop.multiProcessorCount > 0)
      ncu = prop.multiProcessorCount;
  }
  c->m_occ = occ;
  c->m_ncu = ncu;
  {
    const srm_status st = apply_tuning(c, default_tuning(P));
    if (st != SRM_OK) return bail(st);
  }

  // Host tables and the starting state: rho_i^2 = 1, Sigma_s = I, P_i = I.
  Scalars sc{};
  std::vector<double> ones(P.N, 1.0);
  std::vector<double> eyeKP((size_t)P.KP * P.KP, 0.0);
  for (int j = 0; j < P.k; ++j) eyeKP[(size_t)j * P.KP + j] = 1.0;
  std::vector<double> pI((size_t)P.N * P.KP * P.KP, 0.0);
  for (int i = 0; i < P.N; ++i)
    for (int j = 0; j < P.k; ++j) pI[((size_t)i * P.KP + j) * P.KP + j] = 1.0;
  auto up = [&](size_t off, const void* src, size_t n) {
    return hipMemcpyAsync(c->ws + off, src, n, hipMemcpyHostToDevice, c->stream);
  };
  if (up(P.o_sc, &sc, sizeof sc) != hipSuccess ||
      up(P.o_rho2, ones.data(), sizeof(double) * P.N) != hipSuccess ||
      up(P.o_sigcur, eyeKP.data(), eyeKP.size() * 8) != hipSuccess ||
      up(P.o_p64, pI.data(), pI.size() * 8) != hipSuccess ||
      hipStreamSynchronize(c->stream) != hipSuccess)
    return bail(fail(SRM_E_HIP, "upload of tables failed"));
  *out = c;
  return SRM_OK;
}

srm_status srm_ingest(srm_ctx* c, int32_t i, const float* X_i, const double* W0_i) {
  if (!c) return fail(SRM_E_ARG, "ctx is NULL");
  if (c->ready) return fail(SRM_E_STATE, "srm_init_end has already completed");
  const Plan& P = c->p;
  if (i < 0 || i >= P.N) return fail(SRM_E_ARG, "subject %d out of range", i);
  if (!X_i) return fail(SRM_E_ARG, "X[%d] is NULL", i);
  if (c->ingested[i]) return fail(SRM_E_ARG, "subject %d was already ingested", i);
  const Subject& su = P.subj[i];
  if (W0_i) {
    if (!(c->flags & SRM_NO_W0_CHECK) && !c->w0_checked) {
      const double err = w0_error(W0_i, su.v, P.k);
      if (!(err <= 1e-8))
        return fail(SRM_E_ARG, "W0[%d] is not orthonormal (max|W^T W - I| = %g)", i, err);
    }
    const srm_status s = upload_w0(c, i, W0_i);
    if (s != SRM_OK) return s;
  } else {
    SeedArgs sa{c->ws + P.o_arec,
                c->ws + P.o_arec + (P.prec == SRM_FP32 ? 0 : P.arec_bytes / 2), su.row0,
                su.v, su.vp, P.k, i, c->seed, P.prec};
    HIP_OR_FAIL(launch_seed(c->stream, P.KP, sa));
  }
  if (c->flags & SRM_X_HOST) {
    // Streamed ingestion: chunks of the subject's FP32 rows alternate between
    // two staging buffers.  Uploads run on the copy stream, conversions on
    // the compute stream; events order each buffer's reuse.
    for (int64_t r0 = 0; r0 < su.v; r0 += P.stage_rows) {
      const int64_t n = std::min<int64_t>(P.stage_rows, su.v - r0);
      const int b = (int)(c->stage_seq++ & 1);
      float* stage = c->at<float>(P.o_stage + b * P.stage_bytes);
      HIP_OR_FAIL(hipStreamWaitEvent(c->cstream, c->ev_conv[b], 0));
      HIP_OR_FAIL(hipMemcpyAsync(stage, X_i + r0 * P.t, (size_t)(n * P.t) * sizeof(float),
                                 hipMemcpyHostToDevice, c->cstream));
      HIP_OR_FAIL(hipEventRecord(c->ev_up[b], c->cstream));
      HIP_OR_FAIL(hipStreamWaitEvent(c->stream, c->ev_up[b], 0));
      HIP_OR_FAIL(convert_rows(c, i, stage, r0, n, r0 + n >= su.v));
      HIP_OR_FAIL(hipEventRecord(c->ev_conv[b], c->stream));
    }
    // The caller may free or reuse X_i once this returns.
    HIP_OR_FAIL(hipStreamSynchronize(c->cstream));
  } else {
    HIP_OR_FAIL(convert_rows(c, i, X_i, 0, su.v, true));
    // The caller may free or reuse X_i once this returns.
    HIP_OR_FAIL(hipStreamSynchronize(c->stream));
  }
  c->ingested[i] = 1;
  c->seeded[i] = W0_i ? 0 : 1;
  return SRM_OK;
}

srm_status srm_init_end(srm_ctx* c) {
  if (!c) return fail(SRM_E_ARG, "ctx is NULL");
  if (c->ready) return fail(SRM_E_STATE, "srm_init_end has already completed");
  const Plan& P = c->p;
  for (int i = 0; i < P.N; ++i)
    if (!c->ingested[i]) return fail(SRM_E_STATE, "subject %d has not been ingested", i);
  if (launch_rowsum(c->stream, P.N, c->at<double>(P.o_rowc), c->at<Subject>(P.o_subj),
                    c->at<double>(P.o_c)) != hipSuccess)
    return fail(SRM_E_HIP, "conversion launch failed");
  Scalars chk{};
  HIP_OR_FAIL(hipMemcpyAsync(&chk, c->ws + P.o_sc, sizeof chk, hipMemcpyDeviceToHost,
                             c->stream));
  HIP_OR_FAIL(hipStreamSynchronize(c->stream));
  if (chk.nonfinite) return fail(SRM_E_NONFINITE, "X contains NaN or Inf");

  if (P.gram) {
    // Per-subject sample Gram matrices, and a subject table in which subject
    // i's E-phase partial is slice i (the sample-space iteration writes one).
    std::vector<Subject> sg(P.subj);
    for (int i = 0; i < P.N; ++i) {
      sg[i].s_beg = i;
      sg[i].s_end = i + 1;
    }
    HIP_OR_FAIL(hipMemcpyAsync(c->ws + P.o_subjg, sg.data(), sizeof(Subject) * P.N,
                               hipMemcpyHostToDevice, c->stream));
    HIP_OR_FAIL(hipStreamSynchronize(c->stream));
    const Ptrs q = ptrs(c);
    const int nt = (int)(P.ldt / 64);
    const bool g64 = P.prec == SRM_FP32;
    GBArgs gb{q.xh, q.xl, c->at<Subject>(P.o_subj), g64 ? nullptr : c->at<float>(P.o_G),
              g64 ? c->at<double>(P.o_G) : nullptr, P.ldt, nt};
    HIP_OR_FAIL(launch_gram_build(c->stream, P.prec, nt * (nt + 1) / 2, P.N, gb));
  }

  // First E-step with rho^2 = 1, Sigma_s = I and W_i = W0_i (P_i = I), or,
  // where the library drew the start, W_i = polar factor of the drawn
  // Gaussian (P_i = (G_i^T G_i)^-1/2, taken here for every subject).
  bool any_seeded = false;
  for (int i = 0; i < P.N; ++i) any_seeded |= c->seeded[i] != 0;
  if (enqueue_estep(c, false, true, any_seeded) != hipSuccess)
    return fail(SRM_E_HIP, "first E-step launch failed");
  const srm_status s = read_scalars(c, &chk);
  if (s != SRM_OK) return s;
  c->ready = true;
  if (c->flags & SRM_AUTOTUNE) {
    // Launch shapes: from the on-disk cache for this problem and device, else
    // by timed trials (which leave the state as the first E-step left it).
    srm_tuning t{};
    if (tune_cache_find(c, &t) && apply_tuning(c, t) == SRM_OK) return SRM_OK;
    const srm_status st = srm_autotune(c, 2, nullptr, nullptr);
    if (st != SRM_OK) {
      c->ready = false;
      return st;
    }
  }
  return SRM_OK;
}

srm_status srm_init(srm_ctx** out, const srm_desc* desc, const float* const* X,
                    const double* const* W0, uint64_t seed, void* workspace, size_t ws_bytes) {
  if (!out) return fail(SRM_E_ARG, "out is NULL");
  *out = nullptr;
  Plan p;
  srm_status s = make_plan(desc, p);
  if (s != SRM_OK) return s;
  if (!X) return fail(SRM_E_ARG, "X is NULL");
  for (int i = 0; i < p.N; ++i)
    if (!X[i]) return fail(SRM_E_ARG, "X[%d] is NULL", i);
  if (!workspace) return fail(SRM_E_WORKSPACE, "workspace is NULL");
  if (((uintptr_t)workspace & 255) != 0)
    return fail(SRM_E_WORKSPACE, "workspace must be 256-byte aligned");
  if (ws_bytes < p.total)
    return fail(SRM_E_WORKSPACE, "workspace has %zu bytes, %zu needed", ws_bytes, p.total);
  if (W0 && !(desc->flags & SRM_NO_W0_CHECK)) {  // all maps checked before any device call
    std::vector<double> err(p.N, 0.0);
    for (int i = 0; i < p.N; ++i)
      if (W0[i]) err[i] = w0_error(W0[i], p.subj[i].v, p.k);
    for (int i = 0; i < p.N; ++i)
      if (!(err[i] <= 1e-8))
        return fail(SRM_E_ARG, "W0[%d] is not orthonormal (max|W^T W - I| = %g)", i, err[i]);
  }
  srm_ctx* c = nullptr;
  s = srm_init_begin(&c, desc, seed, workspace, ws_bytes);
  if (s != SRM_OK) return s;
  c->w0_checked = true;
  for (int i = 0; i < p.N && s == SRM_OK; ++i)
    s = srm_ingest(c, i, X[i], W0 ? W0[i] : nullptr);
  if (s == SRM_OK) s = srm_init_end(c);
  if (s != SRM_OK) {
    const std::string msg = g_err;
    srm_free(c);
    g_err = msg;
    return s;
  }
  *out = c;
  return SRM_OK;
}

srm_status srm_em_step(srm_ctx* c, double* loglik) {
  return srm_fit(c, 1, loglik);
}

srm_status srm_fit(srm_ctx* c, int32_t n_iter, double* loglik) {
  srm_status s = check_ready(c);
  if (s != SRM_OK) return s;
  if (n_iter < 0) return fail(SRM_E_ARG, "n_iter < 0");
  if (n_iter == 0) return SRM_OK;
  const int first = c->iters;
  HIP_OR_FAIL(copy_state_regions(c, true));
  s = run_iterations(c, n_iter);
  if (s != SRM_OK) return s;
  Scalars sc{};
  s = read_scalars(c, &sc);
  if (s == SRM_E_RANK || s == SRM_E_NOTPD) return undo_failed_call(c, first, s);
  if (s != SRM_OK) return s;
  if (loglik) {
    // LL index j belongs to the parameters entering iteration j.
    for (int it = 0; it < n_iter; ++it) {
      const int idx = (first + it) & (kLLCapacity - 1);
      HIP_OR_FAIL(hipMemcpy(loglik + it, c->ws + c->p.o_ll + sizeof(double) * idx,
                            sizeof(double), hipMemcpyDeviceToHost));
    }
  }
  return SRM_OK;
}

// The fused sweep never writes A = Xhat S^T to HBM; recompute subject i's
// rows from the current S before W_i = A_i P_i is formed.
static srm_status ensure_a(srm_ctx* c, int i) {
  if (c->a_valid) return SRM_OK;
  const Plan& p = c->p;
  const Ptrs q = ptrs(c);
  const Subject& su = p.subj[i];
  const int64_t nt = (su.vp + 63) / 64;
  const int64_t tpw = 4;
  MArgs ma{q.xh, q.xl, q.shc, q.slc, q.ah, q.al, p.ldt, su.row0, su.row0 + su.vp, nt, tpw,
           c->at<Scalars>(p.o_sc)};
  HIP_OR_FAIL(launch_mphase(c->stream, p.KP, p.prec, (int)((nt + tpw - 1) / tpw), ma));
  return SRM_OK;
}

srm_status srm_profile(srm_ctx* c, int32_t n_iter, double* ms) {
  srm_status s = check_ready(c);
  if (s != SRM_OK) return s;
  if (n_iter < 0 || !ms) return fail(SRM_E_ARG, "invalid argument");
  for (int i = 0; i < SRM_NPHASE; ++i) ms[i] = 0.0;
  for (int i = 0; i < 2 * SRM_NPHASE; ++i)
    if (!c->ev[i]) HIP_OR_FAIL(hipEventCreate(&c->ev[i]));
  const int first = c->iters;
  HIP_OR_FAIL(copy_state_regions(c, true));
  c->profiling = true;
  for (int it = 0; it < n_iter; ++it) {
    for (auto& r : c->recorded) r = false;
    const hipError_t e = enqueue_iteration(c);
    if (e != hipSuccess) {
      c->profiling = false;
      return fail(SRM_E_HIP, "launch failed: %s", hipGetErrorString(e));
    }
    ++c->iters;
    HIP_OR_FAIL(hipStreamSynchronize(c->stream));
    for (int ph = 0; ph < SRM_NPHASE; ++ph) {
      if (!c->recorded[ph]) continue;
      float t = 0.f;
      HIP_OR_FAIL(hipEventElapsedTime(&t, c->ev[2 * ph], c->ev[2 * ph + 1]));
      ms[ph] += t;
    }
  }
  c->profiling = false;
  Scalars sc{};
  s = read_scalars(c, &sc);
  if (s == SRM_E_RANK || s == SRM_E_NOTPD) return undo_failed_call(c, first, s);
  return s;
}

// S_out[:, 0:tn] = W_i^T (X[:, 0:tn] - mu_i 1^T), X with row stride ldx and
// S_out with row stride ldo; column chunks through the E-phase partial buffer.
// Subject i's A rows must be current (ensure_a).
static srm_status transform_cols(srm_ctx* c, int32_t i, const float* X, int64_t ldx,
                                 int64_t ncols, float* S_out, int64_t ldo) {
  const Plan& p = c->p;
  const Subject& su = p.subj[i];
  const Ptrs q = ptrs(c);
  const int64_t cap = (int64_t)(p.zpart_bytes / ((size_t)p.KP * 4));
  const int nsplit = (int)std::max<int64_t>(1, std::min<int64_t>(
      std::min<int64_t>(64, (su.v + 2047) / 2048), cap / 64));
  const int64_t chunk = std::max<int64_t>(64, std::min<int64_t>(
      round_up(ncols, 64), cap / nsplit / 64 * 64));
  if (chunk * nsplit > cap) return fail(SRM_E_WORKSPACE, "transform scratch too small");
  const int rps = (int)((su.v + nsplit - 1) / nsplit);
  for (int64_t c0 = 0; c0 < ncols; c0 += chunk) {
    const int64_t tn = std::min(chunk, ncols - c0);
    TArgs ta{q.ah, q.al, c->at<double>(p.o_mu), c->at<double>(p.o_isd), X + c0, c->at<float>(p.o_zpart),
             su.row0, tn, ldx, su.v, rps, p.prec};
    TFArgs tf{c->at<float>(p.o_zpart), c->at<double>(p.o_p64) + (size_t)i * p.KP * p.KP,
              S_out + c0, tn, ldo, nsplit, p.k};
    HIP_OR_FAIL(launch_transform(c->stream, p.KP, nsplit, ta, tf));
  }
  return SRM_OK;
}

srm_status srm_transform(srm_ctx* c, int32_t i, const float* X_new, int64_t t_new,
                         float* S_out) {
  srm_status s = check_ready(c);
  if (s != SRM_OK) return s;
  const Plan& p = c->p;
  if (i < 0 || i >= p.N) return fail(SRM_E_ARG, "subject %d out of range", i);
  if (!X_new || !S_out) return fail(SRM_E_ARG, "NULL buffer");
  if (t_new < 1) return fail(SRM_E_ARG, "t_new must be >= 1");
  if (c->iters < 1) return fail(SRM_E_STATE, "no iteration has run yet");
  const srm_status sa = ensure_a(c, i);
  if (sa != SRM_OK) return sa;
  return transform_cols(c, i, X_new, t_new, t_new, S_out, t_new);
}

srm_status srm_transform_static(srm_ctx* c, int32_t i, const float* X_new, int64_t t_new,
                                float* S_out) {
  srm_status s = check_ready(c);
  if (s != SRM_OK) return s;
  const Plan& p = c->p;
  if (i < 0 || i >= p.N) return fail(SRM_E_ARG, "subject %d out of range", i);
  if (!X_new || !S_out) return fail(SRM_E_ARG, "NULL buffer");
  if (t_new < 1) return fail(SRM_E_ARG, "t_new must be >= 1");
  if (c->iters < 1) return fail(SRM_E_STATE, "no iteration has run yet");
  void* scr = static_scratch_ptr(c->device);
  if (c->scratch_err != hipSuccess || !scr)
    return fail(SRM_E_HIP, "static scratch unavailable on device %d: %s", c->device,
                hipGetErrorString(c->scratch_err));
  // One launch pair over all t_new columns: one row split needs KP t_new
  // floats of the static scratch; more splits are used while they fit.
  const size_t cap = static_scratch_bytes() / sizeof(float);
  const size_t per_split = (size_t)p.KP * (size_t)t_new;
  if (per_split > cap)
    return fail(SRM_E_ARG,
                "t_new=%lld needs %zu bytes of static scratch at k padded to %d; the maximum "
                "is %zu bytes (t_new <= %zu)", (long long)t_new, per_split * sizeof(float), p.KP,
                static_scratch_bytes(), cap / p.KP);
  const Subject& su = p.subj[i];
  const int nsplit = (int)std::max<int64_t>(1, std::min<int64_t>(
      std::min<int64_t>(64, (su.v + 2047) / 2048), (int64_t)(cap / per_split)));
  const srm_status sa = ensure_a(c, i);
  if (sa != SRM_OK) return sa;
  const Ptrs q = ptrs(c);
  float* part = static_cast<float*>(scr);
  const int rps = (int)((su.v + nsplit - 1) / nsplit);
  TArgs ta{q.ah, q.al, c->at<double>(p.o_mu), c->at<double>(p.o_isd), X_new, part, su.row0,
           t_new, t_new, su.v, rps, p.prec};
  TFArgs tf{part, c->at<double>(p.o_p64) + (size_t)i * p.KP * p.KP, S_out, t_new, t_new,
            nsplit, p.k};
  HIP_OR_FAIL(launch_transform(c->stream, p.KP, nsplit, ta, tf));
  return SRM_OK;
}

srm_status srm_map(srm_ctx* c, int32_t i, int32_t j, const float* X_new, int64_t t_new,
                   float* Y_out) {
  srm_status s = check_ready(c);
  if (s != SRM_OK) return s;
  const Plan& p = c->p;
  if (i < 0 || i >= p.N || j < 0 || j >= p.N) return fail(SRM_E_ARG, "subject out of range");
  if (!X_new || !Y_out) return fail(SRM_E_ARG, "NULL buffer");
  if (t_new < 1) return fail(SRM_E_ARG, "t_new must be >= 1");
  if (c->iters < 1) return fail(SRM_E_STATE, "no iteration has run yet");
  // S_new = W_i^T (X_new - mu_i) in column chunks held in the Y-group
  // scratch (free between iterations), then Y = A_j (P_j S_new).
  // S_new chunks (k rows of float) in the Y-group buffer (ngrp KP ldt
  // doubles): at least 2 ldt >= 128 columns per chunk.
  const size_t cap_cols = (size_t)p.ngrp * p.KP * p.ldt * 8 / ((size_t)p.k * 4) / 64 * 64;
  if (cap_cols < 64) return fail(SRM_E_WORKSPACE, "map scratch too small");
  float* sbuf = c->at<float>(p.o_ygrp);
  srm_status sa = ensure_a(c, i);
  if (sa == SRM_OK && j != i) sa = ensure_a(c, j);
  if (sa != SRM_OK) return sa;
  const Ptrs q = ptrs(c);
  for (int64_t c0 = 0; c0 < t_new; c0 += (int64_t)cap_cols) {
    const int64_t tn = std::min<int64_t>((int64_t)cap_cols, t_new - c0);
    sa = transform_cols(c, i, X_new + c0, t_new, tn, sbuf, tn);
    if (sa != SRM_OK) return sa;
    MapArgs ma{q.ah, q.al, c->at<double>(p.o_p64) + (size_t)j * p.KP * p.KP, sbuf,
               Y_out + c0, p.subj[j].row0, tn, tn, t_new, p.subj[j].v, p.k, p.prec};
    HIP_OR_FAIL(launch_map(c->stream, p.KP, ma));
  }
  return SRM_OK;
}

srm_status srm_get_w(srm_ctx* c, int32_t i, float* dst) {
  srm_status s = check_ready(c);
  if (s != SRM_OK) return s;
  const Plan& p = c->p;
  if (i < 0 || i >= p.N) return fail(SRM_E_ARG, "subject %d out of range", i);
  if (!dst) return fail(SRM_E_ARG, "dst is NULL");
  if (c->iters < 1) return fail(SRM_E_STATE, "no iteration has run yet");
  const Ptrs q = ptrs(c);
  srm_status sa = ensure_a(c, i);
  if (sa != SRM_OK) return sa;
  WArgs wa{q.ah, q.al, c->at<double>(p.o_p64) + (size_t)i * p.KP * p.KP, dst,
           p.subj[i].row0, p.subj[i].v, p.k, p.prec};
  HIP_OR_FAIL(launch_get_w(c->stream, p.KP, wa));
  return SRM_OK;
}

srm_status srm_get_s(srm_ctx* c, float* dst) {
  srm_status s = check_ready(c);
  if (s != SRM_OK) return s;
  if (!dst) return fail(SRM_E_ARG, "dst is NULL");
  if (c->iters < 1) return fail(SRM_E_STATE, "no iteration has run yet");
  const Plan& p = c->p;
  std::vector<double> sv((size_t)p.KP * p.ldt);
  HIP_OR_FAIL(hipMemcpyAsync(sv.data(), c->ws + p.o_s64cur, sv.size() * 8,
                             hipMemcpyDeviceToHost, c->stream));
  HIP_OR_FAIL(hipStreamSynchronize(c->stream));
  std::vector<float> f((size_t)p.k * p.t);
  for (int j = 0; j < p.k; ++j)
    for (int64_t col = 0; col < p.t; ++col)
      f[(size_t)j * p.t + col] = (float)sv[(size_t)j * p.ldt + col];
  HIP_OR_FAIL(hipMemcpyAsync(dst, f.data(), f.size() * 4, hipMemcpyHostToDevice, c->stream));
  HIP_OR_FAIL(hipStreamSynchronize(c->stream));
  return SRM_OK;
}

srm_status srm_get_rho2(srm_ctx* c, double* dst) {
  srm_status s = check_ready(c);
  if (s != SRM_OK) return s;
  if (!dst) return fail(SRM_E_ARG, "dst is NULL");
  HIP_OR_FAIL(hipMemcpyAsync(dst, c->ws + c->p.o_rho2, sizeof(double) * c->p.N,
                             hipMemcpyDeviceToHost, c->stream));
  HIP_OR_FAIL(hipStreamSynchronize(c->stream));
  return SRM_OK;
}

srm_status srm_get_sigma_s(srm_ctx* c, double* dst) {
  srm_status s = check_ready(c);
  if (s != SRM_OK) return s;
  if (!dst) return fail(SRM_E_ARG, "dst is NULL");
  if (c->iters < 1) return fail(SRM_E_STATE, "no iteration has run yet");
  const Plan& p = c->p;
  std::vector<double> sv((size_t)p.KP * p.KP);
  HIP_OR_FAIL(hipMemcpyAsync(sv.data(), c->ws + p.o_sigcur, sv.size() * 8,
                             hipMemcpyDeviceToHost, c->stream));
  HIP_OR_FAIL(hipStreamSynchronize(c->stream));
  for (int a = 0; a < p.k; ++a)
    for (int b = 0; b < p.k; ++b) dst[(size_t)a * p.k + b] = sv[(size_t)a * p.KP + b];
  return SRM_OK;
}

srm_status srm_get_mu(srm_ctx* c, int32_t i, double* dst) {
  srm_status s = check_ready(c);
  if (s != SRM_OK) return s;
  if (i < 0 || i >= c->p.N) return fail(SRM_E_ARG, "subject %d out of range", i);
  if (!dst) return fail(SRM_E_ARG, "dst is NULL");
  HIP_OR_FAIL(hipMemcpyAsync(dst, c->ws + c->p.o_mu + sizeof(double) * c->p.subj[i].row0,
                             sizeof(double) * c->p.subj[i].v, hipMemcpyDeviceToDevice,
                             c->stream));
  return SRM_OK;
}

srm_status srm_get_scale(srm_ctx* c, int32_t i, double* dst) {
  srm_status s = check_ready(c);
  if (s != SRM_OK) return s;
  if (i < 0 || i >= c->p.N) return fail(SRM_E_ARG, "subject %d out of range", i);
  if (!dst) return fail(SRM_E_ARG, "dst is NULL");
  HIP_OR_FAIL(hipMemcpyAsync(dst, c->ws + c->p.o_isd + sizeof(double) * c->p.subj[i].row0,
                             sizeof(double) * c->p.subj[i].v, hipMemcpyDeviceToDevice,
                             c->stream));
  return SRM_OK;
}

srm_status srm_get_state(srm_ctx* c, void* blob, size_t* bytes) {
  if (!c) return fail(SRM_E_ARG, "ctx is NULL");
  if (!bytes) return fail(SRM_E_ARG, "bytes is NULL");
  const Plan& p = c->p;
  const size_t need = state_bytes(p);
  if (!blob) {
    *bytes = need;
    return SRM_OK;
  }
  if (*bytes < need) {
    *bytes = need;
    return fail(SRM_E_ARG, "state blob needs %zu bytes", need);
  }
  const srm_status s = check_ready(c);
  if (s != SRM_OK) return s;
  const StateHeader h = make_header(c);
  char* out = static_cast<char*>(blob);
  std::memcpy(out, &h, sizeof(h));
  size_t pos = sizeof(h);
  HIP_OR_FAIL(hipMemcpyAsync(out + pos, c->ws + p.o_c, sizeof(double) * p.N,
                             hipMemcpyDeviceToHost, c->stream));
  pos += sizeof(double) * p.N;
  for (const auto& r : state_regions(p)) {
    HIP_OR_FAIL(hipMemcpyAsync(out + pos, c->ws + r.first, r.second, hipMemcpyDeviceToHost,
                               c->stream));
    pos += r.second;
  }
  HIP_OR_FAIL(hipStreamSynchronize(c->stream));
  *bytes = need;
  return SRM_OK;
}

srm_status srm_set_state(srm_ctx* c, const void* blob, size_t bytes) {
  srm_status s = check_ready(c);
  if (s != SRM_OK) return s;
  if (!blob) return fail(SRM_E_ARG, "blob is NULL");
  const Plan& p = c->p;
  StateHeader h{};
  if (bytes < sizeof(h)) return fail(SRM_E_ARG, "state blob too short");
  std::memcpy(&h, blob, sizeof(h));
  const StateHeader mine = make_header(c);
  if (std::memcmp(h.magic, kStateMagic, 8) != 0 || h.version != kStateVersion)
    return fail(SRM_E_ARG, "not an SRM state blob");
  if (h.N != mine.N || h.k != mine.k || h.KP != mine.KP || h.prec != mine.prec ||
      h.fused != mine.fused || h.t != mine.t || h.ldt != mine.ldt ||
      h.total_rows != mine.total_rows || h.vhash != mine.vhash)
    return fail(SRM_E_ARG, "state blob was taken from a different problem");
  if (h.bytes != mine.bytes || bytes < h.bytes)
    return fail(SRM_E_ARG, "state blob size %zu does not match %llu", bytes,
                (unsigned long long)mine.bytes);
  if (h.iters < 0) return fail(SRM_E_ARG, "state blob holds a negative iteration count");
  const char* in = static_cast<const char*>(blob);
  size_t pos = sizeof(h);
  std::vector<double> cdev(p.N);
  HIP_OR_FAIL(hipMemcpyAsync(cdev.data(), c->ws + p.o_c, sizeof(double) * p.N,
                             hipMemcpyDeviceToHost, c->stream));
  HIP_OR_FAIL(hipStreamSynchronize(c->stream));
  if (std::memcmp(cdev.data(), in + pos, sizeof(double) * p.N) != 0)
    return fail(SRM_E_ARG, "state blob was taken from different data");
  pos += sizeof(double) * p.N;
  for (const auto& r : state_regions(p)) {
    HIP_OR_FAIL(hipMemcpyAsync(c->ws + r.first, in + pos, r.second, hipMemcpyHostToDevice,
                               c->stream));
    pos += r.second;
  }
  HIP_OR_FAIL(hipStreamSynchronize(c->stream));
  c->iters = h.iters;
  c->a_valid = false;  // A = Xhat S^T is rebuilt from S when a getter needs it
  return SRM_OK;
}

srm_status srm_get_loglik(srm_ctx* c, double* dst, int32_t capacity, int32_t* count) {
  srm_status s = check_ready(c);
  if (s != SRM_OK) return s;
  if (!count) return fail(SRM_E_ARG, "count is NULL");
  Scalars sc{};
  HIP_OR_FAIL(hipMemcpyAsync(&sc, c->ws + c->p.o_sc, sizeof sc, hipMemcpyDeviceToHost,
                             c->stream));
  HIP_OR_FAIL(hipStreamSynchronize(c->stream));
  *count = sc.ll_count;
  if (dst) {
    const int n = std::min(std::min(capacity, sc.ll_count), kLLCapacity);
    for (int j = 0; j < n; ++j)
      HIP_OR_FAIL(hipMemcpy(dst + j, c->ws + c->p.o_ll + sizeof(double) * j, sizeof(double),
                            hipMemcpyDeviceToHost));
  }
  return SRM_OK;
}

srm_status srm_get_tuning(const srm_ctx* c, srm_tuning* t) {
  if (!c || !t) return fail(SRM_E_ARG, "NULL argument");
  *t = c->tune;
  return SRM_OK;
}

srm_status srm_set_tuning(srm_ctx* c, const srm_tuning* t) {
  srm_status s = check_ready(c);
  if (s != SRM_OK) return s;
  if (!t) return fail(SRM_E_ARG, "tuning is NULL");
  return apply_tuning(c, *t);
}

srm_status srm_tuning_candidates(const srm_ctx* c, srm_tuning* out, int32_t capacity,
                                 int32_t* count) {
  if (!c || !count) return fail(SRM_E_ARG, "NULL argument");
  const auto all = tuning_candidates(c->p);
  *count = (int32_t)all.size();
  if (out)
    for (int i = 0; i < std::min<int>(capacity, (int)all.size()); ++i) out[i] = all[i];
  return SRM_OK;
}

srm_status srm_autotune(srm_ctx* c, int32_t trials, srm_tuning* best, double* best_ms) {
  srm_status s = check_ready(c);
  if (s != SRM_OK) return s;
  if (trials < 1) return fail(SRM_E_ARG, "trials must be >= 1");
  const srm_tuning start = c->tune;
  const int it0 = c->iters;
  HIP_OR_FAIL(copy_state_regions(c, true));
  const auto all = tuning_candidates(c->p);
  // Coordinate search: the sweep's shapes at the default reduction, then the
  // reduction's shapes at the best sweep.  The current shape is timed first
  // and a candidate replaces the best only when it is faster by more than
  // kTuneMargin, about the spread of repeated trials of one shape.
  constexpr double kTuneMargin = 0.01;
  srm_tuning bt = start;
  double bms = 1e300;
  int bad = 0;
  auto trial = [&](const srm_tuning& t) -> srm_status {
    double ms = 0.0;
    const srm_status st = time_tuning(c, t, trials, &ms, &bad);
    if (st != SRM_OK || bad) return st;
    if (ms < bms * (1.0 - kTuneMargin)) {
      bms = ms;
      bt = t;
    }
    return SRM_OK;
  };
  const int r0 = default_tuning(c->p).reduce_wgs;
  s = trial(start);
  for (const auto& t : all) {
    if (s != SRM_OK || bad) break;
    if (t.reduce_wgs != r0 || same_tuning(t, start)) continue;
    s = trial(t);
  }
  if (s == SRM_OK && !bad) {
    const srm_tuning sw = bt;
    for (const auto& t : all) {
      if (t.reduce_wgs == r0 || t.sweep_kernel != sw.sweep_kernel || t.sweep_wgs != sw.sweep_wgs ||
          t.chunk_rows != sw.chunk_rows || t.mphase_rounds != sw.mphase_rounds)
        continue;
      s = trial(t);
      if (s != SRM_OK || bad) break;
    }
  }
  c->iters = it0;
  c->a_valid = false;  // the trials overwrote the A records
  if (s != SRM_OK || bad) {
    const std::string msg = g_err;
    (void)apply_tuning(c, start);
    g_err = msg;
    if (s != SRM_OK) return s;
    return fail((srm_status)bad, "a trial iteration raised a numeric failure (status %d); "
                "the state is unchanged", bad);
  }
  s = apply_tuning(c, bt);
  if (s != SRM_OK) return s;
  tune_cache_store(c, bt, bms);
  if (best) *best = bt;
  if (best_ms) *best_ms = bms;
  return SRM_OK;
}

srm_status srm_get_info(const srm_ctx* c, srm_info* info) {
  if (!c || !info) return fail(SRM_E_ARG, "NULL argument");
  const Plan& p = c->p;
  std::memset(info, 0, sizeof(*info));
  info->sweep = p.gram ? SRM_SWEEP_GRAM : (p.fused ? SRM_SWEEP_ONE_PASS : SRM_SWEEP_TWO_PASS);
  info->graph = c->graph_used ? 1 : 0;
  info->k_padded = p.KP;
  info->n_ranges = p.nranges;
  info->n_slices = p.nslices;
  info->ldt = p.ldt;
  info->workspace_bytes = p.total;
  return SRM_OK;
}

srm_status srm_iterations(const srm_ctx* c, int32_t* n) {
  if (!c || !n) return fail(SRM_E_ARG, "NULL argument");
  *n = c->iters;
  return SRM_OK;
}

const char* srm_last_error(void) { return g_err.c_str(); }

void srm_free(srm_ctx* c) {
  if (!c) return;
  if (c->stream) (void)hipStreamSynchronize(c->stream);
  if (c->cstream) (void)hipStreamSynchronize(c->cstream);
  for (auto& e : c->ev)
    if (e) (void)hipEventDestroy(e);
  for (int b = 0; b < 2; ++b) {
    if (c->ev_up[b]) (void)hipEventDestroy(c->ev_up[b]);
    if (c->ev_conv[b]) (void)hipEventDestroy(c->ev_conv[b]);
  }
  if (c->gexec) (void)hipGraphExecDestroy(c->gexec);
  if (c->graph) (void)hipGraphDestroy(c->graph);
  if (c->cstream) (void)hipStreamDestroy(c->cstream);
  if (c->own_stream && c->stream) (void)hipStreamDestroy(c->stream);
  delete c;
}

}  // extern "C"
