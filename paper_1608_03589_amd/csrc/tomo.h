// Internal definitions of the tomographic data term: workspace layout and
// the launchers shared by the kernels (tomo.hip) and the C ABI
// (tomo_api.hip).
//
// Operators.  A is the discrete Radon transform with hat weights,
//   (A f)[k][i] = sum_ab f[a][b] max(0, 1 - |x_b cos_k + y_a sin_k - t_i|),
// and A^T its transpose, linear interpolation of each projection in t summed
// over the angles (the backprojection of Section 2, eq. bp_app, without the
// factor pi / n_angles).  Both are gathers:
//
//  * projection (one lane per detector bin, a block of 8 angles by 64
//    bins): for an angle with |cos| >=
//    |sin| the lane walks the image rows; in row a the bin's hat covers the
//    columns within 1/|cos| of j* = (t_i - y_a sin) / cos + (nx - 1) / 2, at
//    most three of them.  For |sin| > |cos| the lane walks the columns of the
//    transposed image instead, so every walk reads rows.  j* advances by the
//    constant -sin/cos per row and is carried in 32.32 fixed point (exact
//    steps; the start is rounded once from float64), so the column index and
//    the weights do not lose bits to the size of j*.  Rows are read from
//    padded copies (kTomoPad zero columns on each side): a wave walks only
//    the rows its bins' hats meet, and in those rows every candidate column
//    of its 64 bins lies inside the padded row, so hats partly outside the
//    image read zeros instead of branching.  The 8 angles of a block walk
//    the same rows (all |cos| >= |sin| or all not) and their 64 bins' hats
//    meet nearby columns, so the block stages a 256-column window of each
//    row in LDS (one 16-byte load per lane and row for the block instead of
//    a 12-byte gather per lane for each angle) and every lane reads its
//    three columns from there; blocks whose angles straddle a diagonal, or
//    whose columns spread wider than the window, gather from memory.
//
//  * backprojection (one lane per pixel, eight pixels per lane down a
//    column): a block owns a 32 x 64 pixel tile; for each angle the tile's
//    projections x cos + y sin span at most 71 bins, and a window of
//    kBpWin bins per angle (as pairs s_i, s_{i+1} - s_i) is staged in LDS
//    for kBpChunk angles at a time.  A pixel's position in its window is
//    formed from the tile corner's (float64, per angle) plus the pixel's
//    small offset (float32), so it keeps about 1e-5 of a bin.
#pragma once

#include "common.h"

namespace tvpd {

constexpr int kTomoPad = 104;        // zero columns on each side of a padded row
constexpr int kTomoMaxSide = 32768;  // ny, nx, n_det limit
constexpr int kTomoMaxAngles = 65535;
constexpr int kProjAngles = 8;       // projection block: 8 angles (one wave
constexpr int kProjThreads = kProjAngles * kWave;  // each) by 64 bins
constexpr int kProjChunk = 16;       // rows staged per round (two per wave)
constexpr int kProjWin = 256;        // staged columns per row (four per lane)
// Column spread of a block's hats in one row that a staged block allows: a
// chunk's window also covers the rows' shift over the chunk (up to one
// column per row), rounding and alignment.
constexpr double kProjMaxSpread = 208.0;
constexpr int kBpRows = 32;          // backprojection tile: rows
constexpr int kBpCols = 64;          //   columns (one wave wide)
constexpr int kBpPerLane = kBpRows / (kMaxBlock / kWave);  // 8 pixels per lane
constexpr int kBpChunk = 32;         // angles staged per round
constexpr int kBpWin = 80;           // bins per staged window (>= 71 + margins)
constexpr int kTomoPrepTile = 32;    // transpose tile of the prep kernel
constexpr int kFbpOut = 8 * 256;     // filtered outputs per block (8 per thread)
constexpr int kFbpIn = 1024;         // inputs staged per round

// Length of the zero-padded filtering grid: the smallest power of two
// >= 2 n_det (so circular convolution equals linear convolution on the
// detector).
__host__ __device__ inline int tomo_fbp_length(int nd) {
  int L = 1;
  while (L < 2 * nd) L *= 2;
  return L;
}

// Device state at the start of a tomography workspace.
struct TomoState {
  int32_t k;         // iteration count of the current iterate
  int32_t pad0[7];
  double red[8];     // reduction results (energies, power iteration)
};
static_assert(sizeof(TomoState) <= 256, "tomo header");

struct TomoLayout {
  int ny, nx, na, nd;
  int pitch_b;        // padded row pitch of the image copy (floats)
  int pitch_t;        // padded row pitch of the transposed copy
  int64_t img;        // floats per dense image plane (multiple of 64)
  int64_t sino;       // floats per sinogram plane (multiple of 64)
  int64_t fb, fbt;    // floats of the padded copies
  int64_t max_partials;
  size_t off_trig;    // double2 per angle
  size_t off_part;    // 2 doubles per partial slot
  size_t off_fbp;     // n_det floats: the filter's impulse response
  size_t off_planes;  // first plane
  size_t bytes;
};

// Plane order after off_planes: image planes F0, F1, PX0, PY0, PX1, PY1, V,
// W; sinogram planes R, S; then FB (ny x pitch_b) and FBT (nx x pitch_t).
enum TomoImg { kTF0 = 0, kTF1, kTPX0, kTPY0, kTPX1, kTPY1, kTV, kTW, kTNumImg };
enum TomoSino { kTR = 0, kTS, kTNumSino };

TomoLayout tomo_layout(int ny, int nx, int na, int nd);

struct TomoPtrs {
  TomoState* st;
  double* trig;       // [na][2]: cos, sin
  double* part;       // partials
  float* fbp;         // filter taps
  float* img[kTNumImg];
  float* sino[kTNumSino];
  float* fb;
  float* fbt;
};
TomoPtrs tomo_ptrs(const TomoLayout& L, void* ws);

// What the projection does with its sums.
enum ProjMode { kProjWrite = 0, kProjDual = 1, kProjResid = 2 };
// What the backprojection does with its sums.
enum BpMode { kBpWrite = 0, kBpTikhonov = 1, kBpTV = 2 };

struct ProjArgs {
  const float* fb;
  const float* fbt;
  const double* trig;
  float* out;         // kProjWrite: A x; kProjDual: r (updated in place)
  const float* g;     // kProjDual, kProjResid
  double* part;       // kProjResid: one slot per block
  float sigma;        // kProjDual
  int ny, nx, na, nd, pitch_b, pitch_t;
  int staged;         // 1: stage image rows in LDS where a block allows it
};

struct BpArgs {
  const float* sino;
  const double* trig;
  float* out;          // kBpWrite: A^T s; otherwise f^{k+1}
  const float* f;      // f^k (kBpTikhonov, kBpTV)
  const float* px;     // p^{k+1} (kBpTV)
  const float* py;
  float tau, lam;
  int ny, nx, na, nd;
};

int launch_tomo_trig(double* trig, int na, hipStream_t s);
// Padded copies of fbar = x + theta (x - x_prev) and of its transpose, and
// with px0 != nullptr the dual update p^{k+1} = P_lam(p^k + sigma grad fbar).
// Ring mode (kptr set): x = slot (k & 1), x_prev = the other slot; p^k is read
// from slot (k & 1) of (px, py) and p^{k+1} written to the other.  Without
// kptr, x0 == x1 is the input and px0 must be null.
int launch_tomo_prep(const TomoLayout& L, const float* x0, const float* x1,
                     const int32_t* kptr, float theta, float* fb, float* fbt,
                     float* px0, float* py0, float* px1, float* py1, float sigma,
                     float lam, hipStream_t s);
int launch_tomo_project(const ProjArgs& a, int mode, hipStream_t s);
int tomo_project_blocks(int na, int nd);
// Ring mode (kptr set, modes other than kBpWrite): a.f / f1, a.out / out1
// and a.px, a.py / px1, py1 are slots 0 / 1 of the image, output and dual
// rings; f^k is read from slot (k & 1), p^{k+1} from the other slot, and
// f^{k+1} written to the other slot.
int launch_tomo_backproject(const BpArgs& a, int mode, const int32_t* kptr,
                            const float* f1, float* out1, const float* px1,
                            const float* py1, hipStream_t s);
// Regularised FBP: taps hs[0, nd) of the filter |nu| / (1 + lam |nu|), and
// q = scale * (hs * g) row by row.
int launch_tomo_fbp_taps(float* hs, int nd, float lam, hipStream_t s);
// Regularised FBP filtering through the FFT (LDS transforms of the BST) for
// padded lengths tomo_fbp_length(nd) <= kFbpFftMaxLen: tw receives the
// length-L twiddle table (8 L bytes), q the filtered sinogram times scale.
constexpr int kFbpFftMaxLen = 4096;
int launch_fbp_fft_filter(const float* g, float* q, float2* tw, int na, int nd, float lam,
                          float scale, hipStream_t s);
int launch_tomo_fbp_filter(const float* g, float* q, const float* hs, int na, int nd,
                           float scale, hipStream_t s);
int launch_tomo_fill(float* p, int64_t n, float v, hipStream_t s);
int launch_tomo_advance(TomoState* st, hipStream_t s);
int launch_tomo_set_k(TomoState* st, int k, hipStream_t s);
// Regulariser partials of x: reg 0 -> sum |grad x|, 1 -> sum x^2.
int launch_tomo_regsum(const float* x, int ny, int nx, int reg, double* part,
                       hipStream_t s);
int tomo_regsum_blocks(int ny, int nx);
// Partials of (<v, w>, |w|^2) over n floats.
int launch_tomo_dot(const float* v, const float* w, int64_t n, double* part,
                    hipStream_t s);
int tomo_dot_blocks(int64_t n);
// *red0 = sum of the first components of partials [first, first + n), and
// *red1 (if not null) of the second components, in a fixed order.
int launch_tomo_reduce(const double* part, int64_t first, int64_t n,
                       double* red0, double* red1, hipStream_t s);
// v = w / sqrt(*nrm2) (v = 0 when *nrm2 == 0).
int launch_tomo_scale(float* v, const float* w, int64_t n, const double* nrm2,
                      hipStream_t s);

}  // namespace tvpd
