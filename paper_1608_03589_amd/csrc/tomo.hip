// HIP kernels of the tomographic data term (see tomo.h for the operators'
// layout in memory and the iteration they serve).
#include <climits>
#include <cmath>

#include "tile2d.h"
#include "tomo.h"

namespace tvpd {
namespace {

using dev::block_sum2;
using dev::dual_arg;
using dev::extrap;
using dev::project2;
using dev::prox_factor;

// Angle table in float64: theta_k = k pi / n_angles.
__global__ void tomo_trig_kernel(double* trig, int na) {
  const int k = blockIdx.x * blockDim.x + threadIdx.x;
  if (k >= na) return;
  const double a = (double)k / (double)na;
  trig[2 * k] = cospi(a);
  trig[2 * k + 1] = sinpi(a);
}

// Word 3 of a raw buffer descriptor for 32-bit loads on CDNA.
constexpr int kBufferWord3 = 0x00020000;

// Ring slots of the iteration: with kptr set, slot (k & 1) holds the
// current iterate; without it both pointers of a pair are the same buffer.
__device__ __forceinline__ int ring_parity(const int32_t* kptr) {
  return kptr ? (*kptr & 1) : 0;
}

struct PrepArgs {
  const float* x0;       // slot 0 / slot 1 of the image ring
  const float* x1;
  const int32_t* kptr;   // current iterate in slot (k & 1); null: x0 == x1
  float theta;
  float* fb;
  float* fbt;
  float* px0;            // dual ring (null: no dual update)
  float* py0;
  float* px1;
  float* py1;
  float sigma, lam;
  int ny, nx, pitch_b, pitch_t;
};

// fbar = x + theta (x - x_prev) of a 32 x 32 tile: written to the padded
// copy, transposed through LDS into the padded transposed copy, and (TV)
// the dual update p^{k+1} = P_lam(p^k + sigma grad fbar) of the tile's
// pixels.  Blocks at the image's edges also write the zero pad columns.
__global__ __launch_bounds__(256) void tomo_prep_kernel(PrepArgs a) {
  __shared__ float tile[kTomoPrepTile][kTomoPrepTile + 1];
  const int tx = threadIdx.x, ty = threadIdx.y;   // 32 x 8
  const int b0 = blockIdx.x * kTomoPrepTile, a0 = blockIdx.y * kTomoPrepTile;
  const int ny = a.ny, nx = a.nx;
  const int par = ring_parity(a.kptr);
  const float* x = par ? a.x1 : a.x0;
  const float* xp = par ? a.x0 : a.x1;
  const float th = a.theta;
  auto fbar = [&](int r, int c) {
    const int64_t o = (int64_t)r * nx + c;
    return extrap(x[o], xp[o], th);
  };
  const bool dual = a.px0 != nullptr;
  const float* pxi = par ? a.px1 : a.px0;
  const float* pyi = par ? a.py1 : a.py0;
  float* pxo = par ? a.px0 : a.px1;
  float* pyo = par ? a.py0 : a.py1;
#pragma unroll
  for (int rr = 0; rr < kTomoPrepTile; rr += 8) {
    const int r = a0 + ty + rr, c = b0 + tx;
    if (r < ny && c < nx) {
      const float v = fbar(r, c);
      a.fb[(int64_t)r * a.pitch_b + kTomoPad + c] = v;
      tile[ty + rr][tx] = v;
      if (dual) {
        const int64_t o = (int64_t)r * nx + c;
        const float gx = c + 1 < nx ? fbar(r, c + 1) - v : 0.0f;
        const float gy = r + 1 < ny ? fbar(r + 1, c) - v : 0.0f;
        float qx, qy;
        project2(dual_arg(pxi[o], a.sigma, gx), dual_arg(pyi[o], a.sigma, gy),
                 a.lam, qx, qy);
        pxo[o] = qx;
        pyo[o] = qy;
      }
    }
    if (r < ny) {
      for (int j = tx; j < kTomoPad; j += kTomoPrepTile) {
        if (blockIdx.x == 0) a.fb[(int64_t)r * a.pitch_b + j] = 0.0f;
        if (blockIdx.x == gridDim.x - 1)
          a.fb[(int64_t)r * a.pitch_b + kTomoPad + nx + j] = 0.0f;
      }
    }
  }
  __syncthreads();
#pragma unroll
  for (int rr = 0; rr < kTomoPrepTile; rr += 8) {
    const int c = b0 + ty + rr, r = a0 + tx;   // row c of the transpose
    if (c < nx && r < ny) a.fbt[(int64_t)c * a.pitch_t + kTomoPad + r] = tile[tx][ty + rr];
    if (c < nx) {
      for (int j = tx; j < kTomoPad; j += kTomoPrepTile) {
        if (blockIdx.y == 0) a.fbt[(int64_t)c * a.pitch_t + j] = 0.0f;
        if (blockIdx.y == gridDim.y - 1)
          a.fbt[(int64_t)c * a.pitch_t + kTomoPad + ny + j] = 0.0f;
      }
    }
  }
}

// Projection: one lane per bin of one angle, a block of kProjAngles angles
// by 64 bins (see tomo.h).
//
// Weights.  With e = j* - rr = jl + phi (jl integer, 0 <= phi < 1) and
// aa = |cos| (rows) or |sin| (columns), aa rr = 1, the hat weights
// 1 - aa |column - j*| of the three candidate columns jl + 1, jl + 2, jl + 3
// reduce to
//     w1 = aa (1 - phi),
//     w2 = 1 - |2 aa - 1 - aa phi|        (in [0, 1] for aa >= 1/sqrt(2)),
//     w3 = max(0, 2 - 3 aa + aa phi).
//
// Rows.  A wave's 64 bins lie within 63 / aa <= 89.1 columns of each other in
// every row; the wave walks only the rows in which at least one of its
// bins' hats meets the image (plus one row on each side), and there every
// candidate column lies inside the padded row (kTomoPad >= 94 zeros; 10
// spare), so no per-row clamp is needed.

// Geometry of one angle for the 64 bins from i0w: the walk's rows, the
// fixed-point column of each bin, and the column range of the 64 bins.
struct ProjAngle {
  bool xmaj;        // walks the rows of the image (else of its transpose)
  double al;        // cos (rows) or sin (columns)
  double m;         // column step per row, -sin/cos or -cos/sin
  double rr;        // half-width of the hat in columns, 1/|al|
  double cq0;       // coordinate of row 0, 1/2 - nq/2
  int q_lo, q_hi;   // rows met (q_hi < q_lo: none)
  double e_lo;      // min over the 64 bins of e at row coordinate 0
  double e_hi;      // max
};

__device__ __forceinline__ double proj_A(const ProjArgs& a, double al, int nj, int bin) {
  return ((double)bin + 0.5 - 0.5 * (double)a.nd) / al + 0.5 * (double)(nj - 1);
}

__device__ __forceinline__ ProjAngle proj_angle(const ProjArgs& a, int k, int i0w) {
  ProjAngle g;
  const double c = a.trig[2 * k], s = a.trig[2 * k + 1];
  g.xmaj = fabs(c) >= fabs(s);
  g.al = g.xmaj ? c : s;
  const double be = g.xmaj ? s : c;
  const int nq = g.xmaj ? a.ny : a.nx, nj = g.xmaj ? a.nx : a.ny;
  g.rr = 1.0 / fabs(g.al);
  // j*(q) = A_i + m c_q, c_q = q + 1/2 - nq/2 the row's coordinate
  g.m = -be / g.al;
  g.cq0 = 0.5 - 0.5 * (double)nq;
  const double Af = proj_A(a, g.al, nj, i0w), Al = proj_A(a, g.al, nj, i0w + kWave - 1);
  const double Alo = fmin(Af, Al), Ahi = fmax(Af, Al);
  const double lo_j = -g.rr, hi_j = (double)(nj - 1) + g.rr;   // j* range that meets
  g.q_lo = 0;
  g.q_hi = nq - 1;
  if (g.m == 0.0) {
    if (!(Ahi > lo_j && Alo < hi_j)) g.q_hi = -1;
  } else {
    // Ahi + m c > lo_j  and  Alo + m c < hi_j
    double c1 = (lo_j - Ahi) / g.m, c2 = (hi_j - Alo) / g.m;
    const double cmin = fmin(c1, c2), cmax = fmax(c1, c2);
    const double qa = floor(cmin - g.cq0) - 1.0, qb = ceil(cmax - g.cq0) + 1.0;
    g.q_lo = (int)fmax(qa, 0.0);
    g.q_hi = (int)fmin(qb, (double)(nq - 1));
  }
  g.e_lo = Alo - g.rr;
  g.e_hi = Ahi - g.rr;
  return g;
}

// min / max over the 8 lanes of a lane group (lanes l, l^1, ..., l^7).
__device__ __forceinline__ int group_min(int v) {
  v = min(v, __shfl_xor(v, 1));
  v = min(v, __shfl_xor(v, 2));
  return min(v, __shfl_xor(v, 4));
}
__device__ __forceinline__ int group_max(int v) {
  v = max(v, __shfl_xor(v, 1));
  v = max(v, __shfl_xor(v, 2));
  return max(v, __shfl_xor(v, 4));
}
__device__ __forceinline__ double group_min(double v) {
  v = fmin(v, __shfl_xor(v, 1));
  v = fmin(v, __shfl_xor(v, 2));
  return fmin(v, __shfl_xor(v, 4));
}
__device__ __forceinline__ float group_min(float v) {
  v = fminf(v, __shfl_xor(v, 1));
  v = fminf(v, __shfl_xor(v, 2));
  return fminf(v, __shfl_xor(v, 4));
}
__device__ __forceinline__ double group_max(double v) {
  v = fmax(v, __shfl_xor(v, 1));
  v = fmax(v, __shfl_xor(v, 2));
  return fmax(v, __shfl_xor(v, 4));
}

template <int MODE>
__global__ __launch_bounds__(kProjThreads) void tomo_project_kernel(ProjArgs a) {
  __shared__ __attribute__((aligned(16))) float win[2][kProjChunk][kProjWin];
  const float* const wflat = &win[0][0][0];
  __shared__ double red[2][kProjAngles];
  const int lane = threadIdx.x & (kWave - 1);
  const int wave = __builtin_amdgcn_readfirstlane(threadIdx.x / kWave);
  // Blocks are dealt to the 8 XCDs in turn; each XCD takes a contiguous run
  // of (bin chunk, angle group) tiles instead, so that blocks sharing its L2
  // stage overlapping windows of the same rows.
  const int nbx = gridDim.x, nbt = gridDim.x * gridDim.y;
  const int bl = blockIdx.y * nbx + blockIdx.x;
  const int q8 = nbt >> 3, r8 = nbt & 7, xcd = bl & 7;
  const int bt = xcd * q8 + min(xcd, r8) + (bl >> 3);
  const int bx = bt % nbx, by = bt / nbx;
  const int g0 = by * kProjAngles;
  const int k = g0 + wave;
  const bool live = k < a.na;
  const int i0w = bx * kWave;
  const int i = i0w + lane;

  // this wave's angle (waves past the last angle walk no rows)
  const ProjAngle P = proj_angle(a, live ? k : a.na - 1, i0w);
  const float* src = P.xmaj ? a.fb : a.fbt;
  const int64_t pitch = P.xmaj ? a.pitch_b : a.pitch_t;
  const int qlo = __builtin_amdgcn_readfirstlane(P.q_lo);
  const int qhi = live ? __builtin_amdgcn_readfirstlane(P.q_hi) : -1;
  // e(q) = j*(q) - rr in 32.32 fixed point, from row qlo
  constexpr double kFx = 4294967296.0;
  const double e0 = proj_A(a, P.al, P.xmaj ? a.nx : a.ny, i) + P.m * P.cq0 - P.rr;
  const int64_t dE = llrint(P.m * kFx);
  const int64_t E0 = llrint(e0 * kFx) + (int64_t)qlo * dE;
  // the 32.32 value as an integer part and a fraction word, stepped with an
  // explicit carry (two 32-bit adds)
  int32_t hi = (int32_t)(E0 >> 32);
  uint32_t lo = (uint32_t)E0;
  const int32_t dhi = (int32_t)(dE >> 32);
  const uint32_t dlo = (uint32_t)dE;
  const float aa = (float)fabs(P.al);
  const float aaf = aa * 2.3283064365386963e-10f;   // aa 2^-32 (phi carried x 2^32)
  const float c2w = 2.0f * aa - 1.0f, c3w = 2.0f - 3.0f * aa;
  float acc = 0.0f;
  // one row: the hat weights of the lane's three columns v0, v1, v2, then
  // the step to the next row
  auto accumulate = [&](float v0, float v1, float v2) {
    const float ph = (float)lo;                       // phi * 2^32
    const float w1 = fmaf(-aaf, ph, aa);
    const float w2 = 1.0f - fabsf(fmaf(-aaf, ph, c2w));
    const float w3 = __builtin_amdgcn_fmed3f(fmaf(aaf, ph, c3w), 0.0f, 1.0f);
    acc = fmaf(w1, v0, acc);
    acc = fmaf(w2, v1, acc);
    acc = fmaf(w3, v2, acc);
    unsigned carry;
    lo = __builtin_addc(lo, dlo, 0u, &carry);
    hi = (int32_t)__builtin_addc((unsigned)hi, (unsigned)dhi, carry, &carry);
  };
  const int row_bytes = (int)(pitch * sizeof(float));
  constexpr uint32_t kOff0 = (kTomoPad + 1) * sizeof(float);

  // The block's angles, angle g0 + (lane & 7) in every lane (the same in
  // every wave, so every decision below is uniform over the block).
  const int kj = min(g0 + (lane & (kProjAngles - 1)), a.na - 1);
  const ProjAngle G = proj_angle(a, kj, i0w);
  const bool inc = g0 + (lane & (kProjAngles - 1)) < a.na && G.q_hi >= G.q_lo;
  const uint64_t maj = __ballot(G.xmaj);
  const bool same = maj == 0 || maj == ~0ull;
  const int Q0 = __builtin_amdgcn_readfirstlane(group_min(inc ? G.q_lo : INT_MAX));
  const int Q1 = __builtin_amdgcn_readfirstlane(group_max(inc ? G.q_hi : INT_MIN));
  // The columns the block's lanes read in row q lie in [min_j lo_j(q),
  // max_j hi_j(q) + 3] with lo_j, hi_j = e_lo, e_hi + m c_q: the spread is
  // convex in q, so its largest value over [Q0, Q1] is at an end.
  auto spread_at = [&](int q) {
    const double cq = (double)q + G.cq0;
    const double l = group_min(inc ? G.e_lo + G.m * cq : INFINITY);
    const double h = group_max(inc ? G.e_hi + G.m * cq : -INFINITY);
    return h - l;
  };
  const bool any = Q1 >= Q0;
  const int staged = __builtin_amdgcn_readfirstlane(
      (a.staged != 0 && same && any &&
       fmax(spread_at(Q0), spread_at(Q1)) < kProjMaxSpread) ? 1 : 0);

  if (staged) {
    // First padded column of the window of the chunk of rows q0 ..
    // q0 + kProjChunk - 1: two columns below the block's leftmost in any of
    // them (the leftmost of an angle is at the first or the last row), on a
    // 16-byte boundary, in float32 (the window leaves room for its
    // rounding).  Uniform, kept in a scalar register.
    const float elo_f = inc ? (float)G.e_lo : INFINITY;
    const float m_f = (float)G.m, cq0_f = (float)G.cq0;
    auto base_of = [&](int q0) {
      const float c0 = (float)q0 + cq0_f;
      const float l = group_min(
          inc ? fminf(fmaf(m_f, c0, elo_f), fmaf(m_f, c0 + (float)(kProjChunk - 1), elo_f))
              : INFINITY);
      // (the opaque step keeps the conversion ahead of the read-first-lane,
      // so the base and the row addresses built on it are scalar values)
      int pbv = ((int)floorf(l) + kTomoPad - 1) & ~3;
      __asm__ volatile("" : "+v"(pbv));
      return __builtin_amdgcn_readfirstlane(pbv);
    };
    typedef unsigned int Row __attribute__((ext_vector_type(4)));
    constexpr int kRowsPerWave = kProjChunk / kProjAngles;
    // this wave's rows q0 + wave + 8 j of the chunk from q0, with the
    // chunk's base pb; rows past Q1 read nothing (an empty buffer range
    // returns zeros)
    auto load_rows = [&](int q0, int pb, Row* v) {
#pragma unroll
      for (int j = 0; j < kRowsPerWave; ++j) {
        const int q = q0 + wave + j * kProjAngles;
        const __amdgpu_buffer_rsrc_t rs = __builtin_amdgcn_make_buffer_rsrc(
            const_cast<float*>(src + (int64_t)min(q, Q1) * pitch), (short)0,
            q <= Q1 ? row_bytes : 0, kBufferWord3);
        // (columns left of the row wrap to large offsets: out of range, zeros)
        const uint32_t off = (uint32_t)(pb + 4 * lane) * (uint32_t)sizeof(float);
        v[j] = __builtin_amdgcn_raw_buffer_load_b128(rs, off, 0, 0);
      }
    };
    auto store_rows = [&](int buf, const Row* v) {
#pragma unroll
      for (int j = 0; j < kRowsPerWave; ++j) {
        float4 t;
        t.x = __uint_as_float(v[j][0]);
        t.y = __uint_as_float(v[j][1]);
        t.z = __uint_as_float(v[j][2]);
        t.w = __uint_as_float(v[j][3]);
        *reinterpret_cast<float4*>(&win[buf][wave + j * kProjAngles][4 * lane]) = t;
      }
    };
    // Chunk ch is read from window buffer ch & 1; its rows were loaded two
    // chunks earlier into one of two register sets, which alternate (the
    // loop is unrolled by two, so no loaded register is moved).
    const int nch = (Q1 - Q0) / kProjChunk + 1;
    int pb0 = base_of(Q0), pb1 = base_of(Q0 + kProjChunk);
    Row ra[kRowsPerWave], rb[kRowsPerWave];
    load_rows(Q0, pb0, ra);
    load_rows(Q0 + kProjChunk, pb1, rb);
    store_rows(0, ra);
    __syncthreads();
    // one chunk: rows qc .. qc + kProjChunk - 1 from buffer buf with base
    // pbc; the rows of chunk ch + 1 (in nxt) go to the other buffer, and the
    // rows of chunk ch + 2 are loaded into cur's registers, whose base
    // replaces pbc
    auto chunk = [&](int ch, int& pbc, Row* cur, Row* nxt) {
      const int qc = Q0 + ch * kProjChunk;
      const int buf = ch & 1;
      const int pb2 = base_of(qc + 2 * kProjChunk);
      load_rows(qc + 2 * kProjChunk, pb2, cur);
      // the element of the window storage holding padded column 0 of the
      // chunk's row 0, in buffer buf
      const int w0 = buf * kProjChunk * kProjWin + (kTomoPad + 1) - pbc;
      // Row r's column hi is read at w0 + r kProjWin + hi: one shift-add on
      // the row's scalar base.  (The opaque steps keep the row base scalar
      // and stop the compiler from deriving each row's address from the
      // previous one's, which costs two more instructions per row.)
      if (qc >= qlo && qc + kProjChunk - 1 <= qhi) {
        // every row of the chunk (one block of code: the reads of later rows
        // can go ahead of the sums of earlier ones)
#pragma unroll
        for (int r = 0; r < kProjChunk; ++r) {
          int rb = (w0 + r * kProjWin) * (int)sizeof(float);   // bytes
          __asm__ volatile("" : "+s"(rb));
          const float* rowp =
              reinterpret_cast<const float*>(reinterpret_cast<const char*>(wflat) + rb) + hi;
          accumulate(rowp[0], rowp[1], rowp[2]);
          __asm__ volatile("" : "+v"(hi));
        }
      } else {
#pragma unroll
        for (int r = 0; r < kProjChunk; ++r) {
          const int q = qc + r;
          if (q >= qlo && q <= qhi) {
            int rb = (w0 + r * kProjWin) * (int)sizeof(float);   // bytes
            __asm__ volatile("" : "+s"(rb));
            const float* rowp =
                reinterpret_cast<const float*>(reinterpret_cast<const char*>(wflat) + rb) + hi;
            accumulate(rowp[0], rowp[1], rowp[2]);
            __asm__ volatile("" : "+v"(hi));
          }
        }
      }
      store_rows(buf ^ 1, nxt);
      __syncthreads();
      pbc = pb2;
    };
    int ch = 0;
    for (; ch + 1 < nch; ch += 2) {
      chunk(ch, pb0, ra, rb);
      chunk(ch + 1, pb1, rb, ra);
    }
    if (ch < nch) chunk(ch, pb0, ra, rb);
  } else {
    // one buffer descriptor per row (scalar work): reads past the row's end
    // return 0 instead of touching the next row
    const char* rowb = reinterpret_cast<const char*>(src + (int64_t)qlo * pitch);
#pragma unroll 8
    for (int q = qlo; q <= qhi; ++q) {
      const __amdgpu_buffer_rsrc_t rs = __builtin_amdgcn_make_buffer_rsrc(
          const_cast<char*>(rowb), (short)0, row_bytes, kBufferWord3);
      const auto v3 =
          __builtin_amdgcn_raw_buffer_load_b96(rs, ((uint32_t)hi << 2) + kOff0, 0, 0);
      accumulate(__uint_as_float(v3[0]), __uint_as_float(v3[1]),
                 __uint_as_float(v3[2]));
      rowb += row_bytes;
    }
  }
  double v = 0.0, unused = 0.0;
  if (live && i < a.nd) {
    const int64_t o = (int64_t)k * a.nd + i;
    if constexpr (MODE == kProjWrite) {
      a.out[o] = acc;
    } else if constexpr (MODE == kProjDual) {
      a.out[o] = fmaf(a.sigma, acc - a.g[o], a.out[o]) * prox_factor(a.sigma);
    } else {
      const double res = (double)acc - (double)a.g[o];
      v = res * res;
    }
  }
  if constexpr (MODE == kProjResid) {
    block_sum2(v, unused, red);
    if (threadIdx.x == 0) {
      const int64_t slot = bt;
      a.part[2 * slot] = v;
      a.part[2 * slot + 1] = 0.0;
    }
  }
}

struct BpKernelArgs {
  BpArgs b;
  const int32_t* kptr;   // ring mode (null: pointers used as given)
  const float* f1;       // slot 1 of the image ring (f in b is slot 0)
  float* out1;           // slot 1 of the output ring
  const float* px1;      // slot 1 of the dual ring
  const float* py1;
};

// Backprojection of a 32 x 64 tile (see tomo.h), with the primal update in
// the epilogue for the iteration's modes.
template <int MODE>
__global__ __launch_bounds__(kMaxBlock) void tomo_backproject_kernel(BpKernelArgs ka) {
  __shared__ float2 win[kBpChunk][kBpWin];
  __shared__ float4 tab[kBpChunk];
  const BpArgs& a = ka.b;
  const int lane = threadIdx.x & (kWave - 1), wave = threadIdx.x / kWave;
  const int b0 = blockIdx.x * kBpCols, a0 = blockIdx.y * kBpRows;
  // centre of the tile's corner pixel (a0, b0)
  const double xr = b0 + 0.5 - 0.5 * (double)a.nx;
  const double yr = a0 + 0.5 - 0.5 * (double)a.ny;
  const double t0 = 0.5 - 0.5 * (double)a.nd;
  const float dx = (float)lane;
  const float dy = (float)(wave * kBpPerLane);
  float acc[kBpPerLane];
#pragma unroll
  for (int m = 0; m < kBpPerLane; ++m) acc[m] = 0.0f;
  for (int kc = 0; kc < a.na; kc += kBpChunk) {
    const int nk = min(kBpChunk, a.na - kc);
    if ((int)threadIdx.x < nk) {
      const int k = kc + threadIdx.x;
      const double c = a.trig[2 * k], s = a.trig[2 * k + 1];
      const double ur = xr * c + yr * s;
      const double umin = ur + fmin(0.0, (kBpCols - 1) * c) + fmin(0.0, (kBpRows - 1) * s);
      // window of bins [ws, ws + kBpWin); the tile's positions u - t0 - ws lie
      // in [2, 74) (the tile spans at most 71 bins)
      const double ws = floor(umin - t0) - 2.0;
      tab[threadIdx.x] = make_float4((float)c, (float)s, (float)(ur - t0 - ws),
                                     __int_as_float((int)ws));
    }
    __syncthreads();
    for (int e = threadIdx.x; e < nk * kBpWin; e += kMaxBlock) {
      const int kk = e / kBpWin, j = e - kk * kBpWin;
      const int bin = __float_as_int(tab[kk].w) + j;
      const float* row = a.sino + (int64_t)(kc + kk) * a.nd;
      const float s0 = (bin >= 0 && bin < a.nd) ? row[bin] : 0.0f;
      const float s1 = (bin + 1 >= 0 && bin + 1 < a.nd) ? row[bin + 1] : 0.0f;
      win[kk][j] = make_float2(s0, s1 - s0);
    }
    __syncthreads();
    for (int kk = 0; kk < nk; ++kk) {
      const float4 T = tab[kk];
      const float vx = fmaf(dx, T.x, fmaf(dy, T.y, T.z));
#pragma unroll
      for (int m = 0; m < kBpPerLane; ++m) {
        const float v = fmaf((float)m, T.y, vx);   // > 0: truncation is floor
        const int idx = (int)v;
        const float w = __builtin_amdgcn_fractf(v);
        const float2 S = win[kk][idx];
        acc[m] += fmaf(w, S.y, S.x);
      }
    }
    __syncthreads();
  }
  const int b = b0 + lane;
  if (b >= a.nx) return;
  const int par = ring_parity(ka.kptr);
  const float* f = par ? ka.f1 : a.f;
  float* out = par ? a.out : ka.out1;     // slot of k + 1
  if (MODE == kBpWrite) out = a.out;
  const float* px = par ? a.px : ka.px1;  // p^{k+1} sits in slot of k + 1
  const float* py = par ? a.py : ka.py1;
  const float itl = MODE == kBpTikhonov ? 1.0f / (1.0f + a.tau * a.lam) : 1.0f;
#pragma unroll
  for (int m = 0; m < kBpPerLane; ++m) {
    const int r = a0 + wave * kBpPerLane + m;
    if (r >= a.ny) break;
    const int64_t o = (int64_t)r * a.nx + b;
    if constexpr (MODE == kBpWrite) {
      out[o] = acc[m];
    } else if constexpr (MODE == kBpTikhonov) {
      out[o] = fmaf(-a.tau, acc[m], f[o]) * itl;
    } else {
      float d = px[o] - (b > 0 ? px[o - 1] : 0.0f);
      d = d + (py[o] - (r > 0 ? py[o - a.nx] : 0.0f));
      out[o] = fmaf(a.tau, d, fmaf(-a.tau, acc[m], f[o]));
    }
  }
}

// Regularised filtered backprojection: the filter's impulse response.
// hs[n] (0 <= n < nd) = (1/L) sum_m H_m cos(2 pi m n / L) with
// H_m = |nu_m| / (1 + lam |nu_m|), nu_m the signed DFT frequency of index m
// on the length-L grid (H is even, so the response is real and even).
// One wave per tap, its lanes striding over m; float64, the product m n
// reduced modulo L exactly before the cosine.
__global__ __launch_bounds__(kMaxBlock) void tomo_fbp_taps_kernel(float* hs, int nd, int L,
                                                                  double lam) {
  const int lane = threadIdx.x & (kWave - 1);
  const int n = blockIdx.x * (kMaxBlock / kWave) + wave_in_block();
  if (n >= nd) return;                       // whole waves
  // L is a power of two: 1/L and 2/L are exact, m n mod L is a mask
  // (m n < L nd / 2 <= 2^30, L < 4 nd)
  static_assert(2LL * kTomoMaxSide * kTomoMaxSide <= (1LL << 31), "fbp taps phase range");
  const double inv_l = 1.0 / (double)L, two_inv_l = 2.0 / (double)L;
  double acc = 0.0;
  for (int m = 1 + lane; m < L / 2; m += kWave) {
    const double nu = (double)m * inv_l;
    const int mn = (m * n) & (L - 1);
    acc += 2.0 * (nu / (1.0 + lam * nu)) * cospi((double)mn * two_inv_l);
  }
  acc = dev::wave_sum(acc);
  if (lane == 0) {
    acc += (0.5 / (1.0 + 0.5 * lam)) * ((n & 1) ? -1.0 : 1.0);   // m = L/2
    hs[n] = (float)(acc / (double)L);
  }
}

// q[k][i] = scale sum_j hs[|i - j|] g[k][j] for one projection k and
// kFbpOut outputs per block: each thread accumulates 8 consecutive outputs
// over blocks of 8 inputs from a 16-tap window (aligned LDS reads); inputs
// and taps are staged kFbpIn inputs at a time.
__global__ __launch_bounds__(kMaxBlock) void tomo_fbp_filter_kernel(
    const float* g, float* q, const float* hs, int nd, float scale) {
  __shared__ __align__(16) float gs[kFbpIn];
  __shared__ __align__(16) float hw[kFbpOut + kFbpIn + 8];
  const int k = blockIdx.y;
  const int I0 = blockIdx.x * kFbpOut;
  const int off = 8 * (int)threadIdx.x;            // i0 - I0
  const float* gr = g + (int64_t)k * nd;
  float acc[8];
#pragma unroll
  for (int u = 0; u < 8; ++u) acc[u] = 0.0f;
  for (int J0 = 0; J0 < nd; J0 += kFbpIn) {
    const int nj = min(kFbpIn, nd - J0);
    // hw[e] = h(d) for d = I0 - J0 - (kFbpIn - 1) + e (zero for |d| >= nd)
    const int dmin = I0 - J0 - (kFbpIn - 1);
    __syncthreads();
    for (int e = threadIdx.x; e < kFbpIn; e += kMaxBlock) gs[e] = e < nj ? gr[J0 + e] : 0.0f;
    for (int e = threadIdx.x; e < kFbpOut + kFbpIn + 8; e += kMaxBlock) {
      const int d = dmin + e, ad = d < 0 ? -d : d;
      hw[e] = ad < nd ? hs[ad] : 0.0f;
    }
    __syncthreads();
    // output u, input jj + t: d - dmin = off + u + (kFbpIn - 1) - jj - t
    //   = (off + kFbpIn - 8 - jj) + (u - t + 7); the window starts at a
    // multiple of 8
    for (int jj = 0; jj < kFbpIn; jj += 8) {
      const float4* w4 = reinterpret_cast<const float4*>(hw + off + kFbpIn - 8 - jj);
      float w[16];
#pragma unroll
      for (int v = 0; v < 4; ++v) {
        const float4 x = w4[v];
        w[4 * v] = x.x;
        w[4 * v + 1] = x.y;
        w[4 * v + 2] = x.z;
        w[4 * v + 3] = x.w;
      }
      const float4 ga = *reinterpret_cast<const float4*>(gs + jj);
      const float4 gb = *reinterpret_cast<const float4*>(gs + jj + 4);
      const float gv[8] = {ga.x, ga.y, ga.z, ga.w, gb.x, gb.y, gb.z, gb.w};
#pragma unroll
      for (int t = 0; t < 8; ++t)
#pragma unroll
        for (int u = 0; u < 8; ++u) acc[u] = fmaf(w[u - t + 7], gv[t], acc[u]);
    }
  }
  float* qr = q + (int64_t)k * nd;
#pragma unroll
  for (int u = 0; u < 8; ++u) {
    const int i = I0 + off + u;
    if (i < nd) qr[i] = acc[u] * scale;
  }
}

__global__ void tomo_fill_kernel(float* p, int64_t n, float v) {
  for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n;
       i += (int64_t)gridDim.x * blockDim.x)
    p[i] = v;
}

__global__ void tomo_advance_kernel(TomoState* st) { st->k += 1; }
__global__ void tomo_set_k_kernel(TomoState* st, int k) { st->k = k; }

constexpr int kRedBlocks = 1024;

// Regulariser partials: reg 0 -> sum |grad x| (float64 differences), 1 ->
// sum x^2.
__global__ __launch_bounds__(kMaxBlock) void tomo_regsum_kernel(const float* x, int ny,
                                                                int nx, int reg,
                                                                double* part) {
  __shared__ double red[2][kMaxBlock / kWave];
  const int64_t n = (int64_t)ny * nx;
  double acc = 0.0, unused = 0.0;
  for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n;
       i += (int64_t)gridDim.x * blockDim.x) {
    const double v = x[i];
    if (reg == 0) {
      const int r = (int)(i / nx), c = (int)(i - (int64_t)r * nx);
      const double gx = c + 1 < nx ? (double)x[i + 1] - v : 0.0;
      const double gy = r + 1 < ny ? (double)x[i + nx] - v : 0.0;
      acc += sqrt(gx * gx + gy * gy);
    } else {
      acc += v * v;
    }
  }
  block_sum2(acc, unused, red);
  if (threadIdx.x == 0) {
    part[2 * blockIdx.x] = acc;
    part[2 * blockIdx.x + 1] = 0.0;
  }
}

__global__ __launch_bounds__(kMaxBlock) void tomo_dot_kernel(const float* v,
                                                             const float* w,
                                                             int64_t n, double* part) {
  __shared__ double red[2][kMaxBlock / kWave];
  double vw = 0.0, ww = 0.0;
  for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n;
       i += (int64_t)gridDim.x * blockDim.x) {
    const double a = v[i], b = w[i];
    vw += a * b;
    ww += b * b;
  }
  block_sum2(vw, ww, red);
  if (threadIdx.x == 0) {
    part[2 * blockIdx.x] = vw;
    part[2 * blockIdx.x + 1] = ww;
  }
}

// One block: fixed-order sums of a range of partials.
__global__ __launch_bounds__(kMaxBlock) void tomo_reduce_kernel(const double* part,
                                                                int64_t first, int64_t n,
                                                                double* red0, double* red1) {
  __shared__ double red[2][kMaxBlock / kWave];
  double a = 0.0, b = 0.0;
  for (int64_t i = threadIdx.x; i < n; i += blockDim.x) {
    a += part[2 * (first + i)];
    b += part[2 * (first + i) + 1];
  }
  block_sum2(a, b, red);
  if (threadIdx.x == 0) {
    *red0 = a;
    if (red1) *red1 = b;
  }
}

__global__ void tomo_scale_kernel(float* v, const float* w, int64_t n,
                                  const double* nrm2) {
  const double q = *nrm2;
  const float sc = q > 0.0 ? (float)(1.0 / sqrt(q)) : 0.0f;
  for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n;
       i += (int64_t)gridDim.x * blockDim.x)
    v[i] = w[i] * sc;
}

int grid_1d(int64_t n) {
  const int64_t b = (n + kMaxBlock - 1) / kMaxBlock;
  return (int)(b < 1 ? 1 : (b > 4096 ? 4096 : b));
}

#define TOMO_LAUNCHED() (hipGetLastError() == hipSuccess ? TVPD_OK : TVPD_ERR_HIP)

}  // namespace

int launch_tomo_trig(double* trig, int na, hipStream_t s) {
  tomo_trig_kernel<<<(na + 255) / 256, 256, 0, s>>>(trig, na);
  return TOMO_LAUNCHED();
}

int launch_tomo_prep(const TomoLayout& L, const float* x0, const float* x1,
                     const int32_t* kptr, float theta, float* fb, float* fbt,
                     float* px0, float* py0, float* px1, float* py1, float sigma,
                     float lam, hipStream_t s) {
  PrepArgs a;
  a.x0 = x0;
  a.x1 = x1;
  a.kptr = kptr;
  a.theta = theta;
  a.fb = fb;
  a.fbt = fbt;
  a.px0 = px0;
  a.py0 = py0;
  a.px1 = px1;
  a.py1 = py1;
  a.sigma = sigma;
  a.lam = lam;
  a.ny = L.ny;
  a.nx = L.nx;
  a.pitch_b = L.pitch_b;
  a.pitch_t = L.pitch_t;
  const dim3 grid((L.nx + kTomoPrepTile - 1) / kTomoPrepTile,
                  (L.ny + kTomoPrepTile - 1) / kTomoPrepTile);
  tomo_prep_kernel<<<grid, dim3(kTomoPrepTile, 8), 0, s>>>(a);
  return TOMO_LAUNCHED();
}

int tomo_project_blocks(int na, int nd) {
  return ((nd + kWave - 1) / kWave) * ((na + kProjAngles - 1) / kProjAngles);
}

int launch_tomo_project(const ProjArgs& a, int mode, hipStream_t s) {
  const dim3 grid((a.nd + kWave - 1) / kWave, (a.na + kProjAngles - 1) / kProjAngles);
  switch (mode) {
    case kProjWrite: tomo_project_kernel<kProjWrite><<<grid, kProjThreads, 0, s>>>(a); break;
    case kProjDual: tomo_project_kernel<kProjDual><<<grid, kProjThreads, 0, s>>>(a); break;
    case kProjResid: tomo_project_kernel<kProjResid><<<grid, kProjThreads, 0, s>>>(a); break;
    default: return TVPD_ERR_INVALID_ARG;
  }
  return TOMO_LAUNCHED();
}

int launch_tomo_backproject(const BpArgs& a, int mode, const int32_t* kptr,
                            const float* f1, float* out1, const float* px1,
                            const float* py1, hipStream_t s) {
  BpKernelArgs ka;
  ka.b = a;
  ka.kptr = kptr;
  ka.f1 = f1;
  ka.out1 = out1;
  ka.px1 = px1;
  ka.py1 = py1;
  const dim3 grid((a.nx + kBpCols - 1) / kBpCols, (a.ny + kBpRows - 1) / kBpRows);
  switch (mode) {
    case kBpWrite: tomo_backproject_kernel<kBpWrite><<<grid, kMaxBlock, 0, s>>>(ka); break;
    case kBpTikhonov: tomo_backproject_kernel<kBpTikhonov><<<grid, kMaxBlock, 0, s>>>(ka); break;
    case kBpTV: tomo_backproject_kernel<kBpTV><<<grid, kMaxBlock, 0, s>>>(ka); break;
    default: return TVPD_ERR_INVALID_ARG;
  }
  return TOMO_LAUNCHED();
}

int launch_tomo_fbp_taps(float* hs, int nd, float lam, hipStream_t s) {
  constexpr int kTapsPerBlock = kMaxBlock / kWave;
  tomo_fbp_taps_kernel<<<(nd + kTapsPerBlock - 1) / kTapsPerBlock, kMaxBlock, 0, s>>>(
      hs, nd, tomo_fbp_length(nd), (double)lam);
  return TOMO_LAUNCHED();
}

int launch_tomo_fbp_filter(const float* g, float* q, const float* hs, int na, int nd,
                           float scale, hipStream_t s) {
  const dim3 grid((nd + kFbpOut - 1) / kFbpOut, na);
  tomo_fbp_filter_kernel<<<grid, kMaxBlock, 0, s>>>(g, q, hs, nd, scale);
  return TOMO_LAUNCHED();
}

int launch_tomo_fill(float* p, int64_t n, float v, hipStream_t s) {
  tomo_fill_kernel<<<grid_1d(n), kMaxBlock, 0, s>>>(p, n, v);
  return TOMO_LAUNCHED();
}

int launch_tomo_advance(TomoState* st, hipStream_t s) {
  tomo_advance_kernel<<<1, 1, 0, s>>>(st);
  return TOMO_LAUNCHED();
}

int launch_tomo_set_k(TomoState* st, int k, hipStream_t s) {
  tomo_set_k_kernel<<<1, 1, 0, s>>>(st, k);
  return TOMO_LAUNCHED();
}

int tomo_regsum_blocks(int ny, int nx) {
  const int64_t b = ((int64_t)ny * nx + kMaxBlock - 1) / kMaxBlock;
  return (int)(b < 1 ? 1 : (b > kRedBlocks ? kRedBlocks : b));
}

int launch_tomo_regsum(const float* x, int ny, int nx, int reg, double* part,
                       hipStream_t s) {
  tomo_regsum_kernel<<<tomo_regsum_blocks(ny, nx), kMaxBlock, 0, s>>>(x, ny, nx, reg, part);
  return TOMO_LAUNCHED();
}

int tomo_dot_blocks(int64_t n) {
  const int64_t b = (n + kMaxBlock - 1) / kMaxBlock;
  return (int)(b < 1 ? 1 : (b > kRedBlocks ? kRedBlocks : b));
}

int launch_tomo_dot(const float* v, const float* w, int64_t n, double* part,
                    hipStream_t s) {
  tomo_dot_kernel<<<tomo_dot_blocks(n), kMaxBlock, 0, s>>>(v, w, n, part);
  return TOMO_LAUNCHED();
}

int launch_tomo_reduce(const double* part, int64_t first, int64_t n, double* red0,
                       double* red1, hipStream_t s) {
  tomo_reduce_kernel<<<1, kMaxBlock, 0, s>>>(part, first, n, red0, red1);
  return TOMO_LAUNCHED();
}

int launch_tomo_scale(float* v, const float* w, int64_t n, const double* nrm2,
                      hipStream_t s) {
  tomo_scale_kernel<<<grid_1d(n), kMaxBlock, 0, s>>>(v, w, n, nrm2);
  return TOMO_LAUNCHED();
}

}  // namespace tvpd
