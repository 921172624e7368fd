// Internal layout shared by the host planner (srm_api.cpp) and the kernels
// (srm_kernels.hip).  Not part of the public ABI.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace srm {

// Rows of every subject are padded to a multiple of 32 (one MFMA K-block in
// the E-phase); TRs to a multiple of 64 (one MFMA K-step pair in the M-phase,
// one wave's column panel in the E-phase).  Padding is zero.
constexpr int kRowPad = 32;
constexpr int kColPad = 64;
constexpr int kMaxK = 128;

// One contiguous run of rows of a single subject handled by one E-phase
// workgroup (a workgroup's equal row range split at subject boundaries).
struct Slice {
  int64_t row0;   // first global (padded) row
  int32_t nrows;  // multiple of 32
  int32_t subj;
};

struct Subject {
  int64_t row0;     // first global row of the subject
  int32_t v;        // true voxel count
  int32_t vp;       // padded row count
  int32_t s_beg;    // its slices [s_beg, s_end)
  int32_t s_end;
};

// Device-resident scalars of the current EM state.
struct Scalars {
  double rho0;          // sum_i rho_i^-2 (Eq. 8)
  double logdet;        // log|I + rho0 Sigma_s|
  double sum_vlogrho;   // sum_i v_i log rho_i^2
  double sum_c_rho;     // sum_i c_i / rho_i^2
  double tau_cur;       // tr(Sigma_s) of the current state
  double tau_new;       // tr(Sigma_s) produced by the latest E-step
  int32_t ll_count;     // log-likelihoods written so far
  int32_t status;       // 0 ok, else an srm_status code raised on the device
  int32_t nonfinite;    // set by the conversion kernel
  int32_t polar_warm;   // stored eigenvectors are a valid warm start
};

constexpr int kLLCapacity = 1 << 16;


// Precision codes (match srm_prec).
enum Prec { P_FP32 = 0, P_BF16 = 1, P_BF16X2 = 2 };

// Kernel argument blocks (passed by value; filled by the host planner).
struct ConvertArgs {
  const float* src;          // FP32 rows of one subject, row stride t
  int64_t src_row0;          // subject-local index of src's first row
  int64_t subj_row0;         // first global row of the subject
  int32_t v;                 // the subject's voxel count
  int64_t t, ldt;
  int64_t row_begin;         // global rows [row_begin, row_end) are converted
  int64_t row_end;
  void* xh;
  void* xl;
  double* mu;
  double* isd;               // per row: 1/std with z-scoring, else 1
  double* rowc;
  Scalars* sc;
  int32_t prec;
  int32_t zscore;
};

// Library-drawn random orthonormal start: subject i's A records hold a
// Philox4x64-10 Gaussian (the polar factor is taken by the first E-step).
struct SeedArgs {
  void* ah;
  void* al;
  int64_t row0;   // first global row of the subject
  int32_t v, vp;
  int32_t k;
  int32_t subj;   // subject index (Philox counter word 1)
  uint64_t seed;  // Philox key word 0
  int32_t prec;
};

struct MArgs {
  const void* xh;
  const void* xl;
  const void* sh;  // S records (hi or FP32)
  const void* sl;  // S records (lo)
  void* ah;        // A records out (hi or FP32)
  void* al;        // A records out (lo)
  int64_t ldt;
  int64_t row_begin;  // rows [row_begin, row_end), multiples of 32
  int64_t row_end;
  int64_t ntiles;     // ceil((row_end - row_begin) / 64)
  int64_t tiles_per_wg;
  const Scalars* sc;  // kernels return at once when sc->status is set
};

struct EArgs {
  const void* xh;
  const void* xl;
  const void* ah;
  const void* al;
  const Slice* slices;
  const int32_t* range_slice;  // [nranges + 1]
  float* zpart;                // [nslices][KP][ldt]
  float* gpart;                // [nslices][KP][KP]
  int64_t ldt;
  int32_t npanel;
  int32_t want_gram;
  const Scalars* sc;
};

struct FusedArgs {
  const void* xh;
  const void* xl;
  const void* sh;              // S records (current)
  const void* sl;
  const Slice* slices;
  const int32_t* range_slice;  // [nranges + 1]
  float* zpart;                // [nslices][KP][ldt]
  float* gpart;                // [nslices][KP][KP]
  int64_t ldt;
  const Scalars* sc;
};

struct RArgs {
  const float* zpart;
  const Subject* subj;
  const double* P64;  // [N][KP][KP]
  const double* rho2;
  double* ygrp;       // [ngrp][KP][ldt]
  int32_t N;
  int32_t gsub;
  int64_t ldt;
  const Scalars* sc;
};

struct PrepArgs {
  const double* rho2;
  const double* c;
  const Subject* subj;
  const double* sig;  // [KP][KP] current Sigma_s
  double* M;          // [KP][KP] out (zero padded)
  Scalars* sc;
  int32_t N;
  int32_t k;
};

struct SArgs {
  const double* ygrp;
  const double* M;
  double* s64;     // [KP][ldt]
  void* sh;        // S records (hi or FP32)
  void* sl;        // S records (lo)
  double* sspart;  // [nblk][KP][KP]
  double* trpart;  // [nblk]
  int32_t ngrp;
  int32_t k;
  int64_t t, ldt;
  const Scalars* sc;
};

struct FinArgs {
  const double* sspart;
  const double* trpart;
  const double* M;
  double* sig_new;
  double* ll;
  Scalars* sc;
  int32_t nblk;
  int32_t k;
  int64_t t;
  double Vtot;
};

struct CopyArgs {
  const double* s64_new;
  double* s64_cur;
  const uint4* srec_new;
  uint4* srec_cur;
  const double* sig_new;
  double* sig_cur;
  Scalars* sc;
  int64_t n_s64;
  int64_t n_srec16;  // in uint4 units
  int32_t n_sig;
};

struct QArgs {
  const float* gpart;
  const Subject* subj;
  const double* c;
  double* rho2;
  double* P64;
  double* work;   // [N][3][KP][KP+1] global scratch (KP > 80)
  double* vprev;  // [N][KP][KP] eigenvectors of the previous iteration
  int32_t* jac;   // [N] 1: Newton-Schulz step not taken (KP > 80, set per launch)
  Scalars* sc;
  int32_t k;
  int64_t t;
  int32_t init_mode;  // 1: polar factor of the drawn start only (rho^2 stays 1)
};

struct WArgs {
  const void* ah;
  const void* al;
  const double* P;  // [KP][KP] of subject i
  float* dst;       // v x k
  int64_t row0;
  int32_t v;
  int32_t k;
  int32_t prec;
};

struct TArgs {
  const void* ah;
  const void* al;
  const double* mu;
  const double* isd;
  const float* X;   // v rows, row stride ldx; columns [0, tn) used
  float* part;      // [nsplit][KP][tn]
  int64_t row0;
  int64_t tn;
  int64_t ldx;
  int32_t v;
  int32_t rows_per_split;
  int32_t prec;
};

struct TFArgs {
  const float* part;
  const double* P;
  float* out;  // k rows, row stride ldo; columns [0, tn)
  int64_t tn;
  int64_t ldo;
  int32_t nsplit;
  int32_t k;
};

struct MapArgs {
  const void* ah;
  const void* al;
  const double* P;   // [KP][KP] of subject j
  const float* s;    // k x tn, row stride lds
  float* out;        // v_j x tn, row stride ldo
  int64_t row0;      // subject j's first global row
  int64_t tn, lds, ldo;
  int32_t v;
  int32_t k;
  int32_t prec;
};

// Sample-space (voxel-free) iteration: G_i = Xhat_i^T Xhat_i, built once.
struct GBArgs {
  const void* xh;
  const void* xl;
  const Subject* subj;
  float* G;         // [N][ldt][ldt] FP32 (BF16 forms), or null
  double* G64;      // [N][ldt][ldt] FP64 (FP32 storage), or null
  int64_t ldt;
  int32_t nt;       // ldt / 64 column tiles
};

// Per iteration: Z_i = S G_i (into the subject's E-phase partial) and the
// per-column-tile partials of Z_i S^T.
struct GZArgs {
  const float* G;     // FP32 G_i (BF16 forms), or null
  const double* G64;  // FP64 G_i (FP32 storage), or null
  const double* S;  // [KP][ldt] FP64 S of the current posterior
  float* zpart;     // [N][KP][ldt]
  double* gz;       // [N][nq][KP][KP]
  int64_t t, ldt;
  int32_t nq;
  int32_t k;
  const Scalars* sc;
};

struct GSArgs {
  const double* gz;
  float* gpart;     // [N][KP][KP]
  int32_t nq;
  const Scalars* sc;
};

}  // namespace srm
