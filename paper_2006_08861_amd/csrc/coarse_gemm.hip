// Coarse screen as one dense product on MFMA with the selection fused into
// its epilogue: the distances from every frame to every region
// representative (the subspace level of the search of Section 3.1) are
// computed tile by tile and never stored. Each lane keeps, per frame it
// holds, the smallest (screen word, region) keys it has seen; only those
// short lists reach memory, and the select kernel then takes the frame's
// best regions from them, re-scores them in FP64 and certifies the choice.
//
// Layout (v_mfma_f32_16x16x32_bf16, A = 16 representatives x 32 dims, B = 32
// dims x 16 frames): a block holds 128 frames, 32 per wave as two 16-frame
// column groups whose bf16 operand (the whole padded length) stays in
// registers for the block's life. Representatives stream through LDS in
// tiles of 32 (two 16-row groups), double-buffered: the next tile is read
// from memory into registers while the current one is multiplied, then
// written to the other buffer. One LDS read of a representative piece feeds
// two MFMAs (the wave's two frame groups).
//
// Lane l of an output tile holds frame l % 16 of its group and
// representatives 4 (l / 16) .. + 3: a quad of four consecutive ones. The
// four lanes l % 16 + 16 g (g = 0..3) share a frame and see disjoint quads.
// Each lane keeps, per frame it holds, the kCgKeep best quads it has seen in
// sorted registers, an entry being (smallest word of the quad << 32 | first
// representative << 4 | slot), the word the float bits of the screen
// distance |q|^2 + |c|^2 - 2 q~.c~ (clamped at 0): entries order by the
// quad's best (distance, representative). A quad entering a list takes the
// memory slot of the entry it pushes out and its four words are stored
// there. A quad left out has its smallest word at or above the list's last
// kept one (the list only improves), so that word bounds every
// representative the list dropped; at the end each lane writes its quads'
// words as (word << 32 | region) keys, and that bound.
#include "hloc_device.h"
#include "hloc_internal.h"

namespace hloc {

typedef float v4f __attribute__((ext_vector_type(4)));
typedef __bf16 v8bf __attribute__((ext_vector_type(8)));
typedef unsigned v4u __attribute__((ext_vector_type(4)));  // 16-byte piece (native vector)

constexpr int kCgWaves = 4;
constexpr int kCgFramesPerWave = 2 * kGroup;              // two MFMA column groups
constexpr int kCgFrames = kCgWaves * kCgFramesPerWave;    // frames per block
constexpr int kCgTile = 32;                               // representatives per LDS tile

// One bf16 representative piece (8 values) against a frame piece.
__device__ __forceinline__ v4f cg_mfma(v4u a, v4u b, v4f acc) {
  return __builtin_amdgcn_mfma_f32_16x16x32_bf16(__builtin_bit_cast(v8bf, a),
                                                 __builtin_bit_cast(v8bf, b), acc, 0, 0, 0);
}

// Inserts e into the ascending list (the last entry falls off the end).
__device__ __forceinline__ void cg_insert(uint64_t (&lst)[kCgKeep], uint64_t e) {
#pragma unroll
  for (int i = 0; i < kCgKeep; ++i) {
    const bool c = lst[i] < e;
    const uint64_t lo = c ? lst[i] : e;
    e = c ? e : lst[i];
    lst[i] = lo;
  }
}

constexpr uint32_t kCgNone = 0xFFFFFFFFu;

// NS = 32-value steps of the padded length (dp / 32), even; LAB: regions
// are restricted to the frame's label.
template <int NS, bool LAB>
__global__ __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(2, 2))) void k_coarse_gemm(
    CoarseGemmArgs a) {
  constexpr int ROWU4 = 4 * NS;      // 16-byte pieces per bf16 row
  constexpr int LDR = ROWU4 + 1;     // pieces per LDS row, one of padding
  constexpr int PER = kCgTile * ROWU4 / 256;  // pieces per thread per tile
  static_assert(kCgTile * ROWU4 % 256 == 0, "whole pieces per thread");
  static_assert(kCgTile <= 256 && (kCgTile & (kCgTile - 1)) == 0, "tile norms by tid bits");
  extern __shared__ v4u s_tile[];  // 2 x kCgTile x LDR
  // (one slot per thread: every thread stores its fetched norm and label,
  // the first kCgTile slots are the tile's)
  __shared__ float s_rn[2][256];
  __shared__ int s_lab[LAB ? 2 : 1][256];

  const int tid = threadIdx.x, lane = lane_id(), w = wave_id();
  const int i = lane & 15, g = lane >> 4;
  const int split = (int)blockIdx.x % a.splits;
  const int f0 = ((int)blockIdx.x / a.splits) * kCgFrames;
  if (f0 >= a.nq) return;
  const int r0 = split * a.reps_per_split;
  const int r1 = min(a.R, r0 + a.reps_per_split);
  const int ntiles = (r1 - r0 + kCgTile - 1) / kCgTile;
  // tiles in a spread order, tile(t) = t * stride mod ntiles with the stride
  // coprime to ntiles (about 5/8 of it): the lists see the whole range early
  // and fill with good quads. In index order the distances along the walk
  // fall toward a frame's own place, and nearly every quad before it would
  // be inserted.
  int stride = 1;
  if (ntiles > 2) {
    stride = (ntiles * 5 / 8) | 1;
    for (;;) {
      int x = stride, y = ntiles;
      while (y) {
        const int t = x % y;
        x = y;
        y = t;
      }
      if (x == 1) break;
      stride += 2;
    }
  }

  const v4u *reps = reinterpret_cast<const v4u *>(a.reps);
  const v4u *frames = reinterpret_cast<const v4u *>(a.frames);

  // the wave's two frame groups: operand and squared norm, and the label a
  // frame's regions must carry
  int fr[2], flab[2];
  float qn[2];
  v4u bv[2][NS];
#pragma unroll
  for (int j = 0; j < 2; ++j) {
    fr[j] = f0 + w * kCgFramesPerWave + j * kGroup + i;
    const int fl = min(fr[j], a.nq - 1);
    qn[j] = a.qn2[fl];
    flab[j] = LAB ? (a.label_frames > 0 ? fl / a.label_frames : a.label) : -1;
#pragma unroll
    for (int s = 0; s < NS; ++s) bv[j][s] = frames[(int64_t)fl * ROWU4 + 4 * s + g];
  }
  // lists: empty entries sort last and carry distinct slots
  uint64_t lst[2][kCgKeep];
#pragma unroll
  for (int j = 0; j < 2; ++j)
#pragma unroll
    for (int e = 0; e < kCgKeep; ++e) lst[j][e] = ~(uint64_t)15 | (uint64_t)e;
  // this lane's quad slots for frame j: slots[slot_base[j] + slot]
  int slot_base[2];  // (nq x splits x 4 x kCgKeep < 2^31: checked by the launcher)
#pragma unroll
  for (int j = 0; j < 2; ++j)
    slot_base[j] = ((min(fr[j], a.nq - 1) * a.splits + split) * 4 + g) * kCgKeep;

  // tile rows are read into registers one tile ahead and written to the
  // other LDS buffer after the current tile is multiplied (indices past r1
  // read the last row; their norm is +inf)
  v4u pv[PER];
  float prn = 0.f;
  int plab = 0;
  // tile t of the order is tile (t stride) mod ntiles: cur_t for the tile
  // multiplied, nxt_t for the one fetched (stride < ntiles, so one step is
  // one conditional subtraction)
  int cur_t = 0, nxt_t = 0;
  auto advance = [&](int x) {
    x += stride;
    return x >= ntiles ? x - ntiles : x;
  };
#define HLOC_CG_FETCH()                                                        \
  {                                                                            \
    const int fb = r0 + nxt_t * kCgTile;                                       \
    _Pragma("unroll") for (int u = 0; u < PER; ++u) {                          \
      const int e = tid + u * 256, row = e / ROWU4, c = e - row * ROWU4;       \
      pv[u] = reps[(int64_t)min(fb + row, r1 - 1) * ROWU4 + c];                \
    }                                                                          \
    {                                                                          \
      const int rr = fb + (tid & (kCgTile - 1));                               \
      const float n2 = a.rep_n2[min(rr, r1 - 1)];                              \
      prn = rr < r1 ? n2 : __builtin_inff();                                   \
      if (LAB) plab = a.rlabel[min(rr, r1 - 1)];                               \
    }                                                                          \
  }
#define HLOC_CG_STAGE(BUF)                                                     \
  {                                                                            \
    _Pragma("unroll") for (int u = 0; u < PER; ++u) {                          \
      const int e = tid + u * 256, row = e / ROWU4, c = e - row * ROWU4;       \
      s_tile[((BUF) * kCgTile + row) * LDR + c] = pv[u];                        \
    }                                                                          \
    s_rn[BUF][tid] = prn;                                                      \
    if (LAB) s_lab[LAB ? (BUF) : 0][tid] = plab;                               \
  }

  if (ntiles > 0) {
    HLOC_CG_FETCH()
    HLOC_CG_STAGE(0)
  }
  // every load so far has landed (the frame operand above all), so the
  // waits inside the loop concern only the next tile's rows
  __builtin_amdgcn_s_waitcnt(0);
  __syncthreads();
  // Every iteration fetches and stages a tile (after the last, tile
  // advance(...) again, never read): with no conditional path the loads
  // are always consumed by the stage, and no wait at the next tile's start
  // holds the epilogue's slot stores.
  for (int t = 0; t < ntiles; ++t) {
    const int buf = t & 1;
    nxt_t = advance(nxt_t);
    HLOC_CG_FETCH()  // in flight while this tile is multiplied
    v4f acc[2][2];
#pragma unroll
    for (int h = 0; h < 2; ++h) {
      acc[h][0] = v4f{0.f, 0.f, 0.f, 0.f};
      acc[h][1] = v4f{0.f, 0.f, 0.f, 0.f};
    }
    const v4u *rp0 = s_tile + (buf * kCgTile + i) * LDR + g;
    const v4u *rp1 = rp0 + kGroup * LDR;
#pragma unroll
    for (int s = 0; s < NS; ++s) {
      const v4u a0 = rp0[4 * s], a1 = rp1[4 * s];
      acc[0][0] = cg_mfma(a0, bv[0][s], acc[0][0]);
      acc[0][1] = cg_mfma(a0, bv[1][s], acc[0][1]);
      acc[1][0] = cg_mfma(a1, bv[0][s], acc[1][0]);
      acc[1][1] = cg_mfma(a1, bv[1][s], acc[1][1]);
    }
    // epilogue: per (row half h, frame group j) the lane's quad of words
    const int base = r0 + cur_t * kCgTile;
#pragma unroll
    for (int h = 0; h < 2; ++h) {
      const int row0 = h * kGroup + 4 * g;
      float rn[4];
      bool rok[4];
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        rn[r] = s_rn[buf][row0 + r];
        rok[r] = !__builtin_isinf(rn[r]);
      }
#pragma unroll
      for (int j = 0; j < 2; ++j) {
        uint32_t wd[4];
#pragma unroll
        for (int r = 0; r < 4; ++r) {
          float dd = (qn[j] + rn[r]) - 2.f * acc[h][j][r];
          dd = dd > 0.f ? dd : 0.f;
          // empty regions (infinite norm), rows past the split and regions
          // outside the frame's label are no candidates
          const bool ok = rok[r] && (!LAB || s_lab[LAB ? buf : 0][row0 + r] == flab[j]);
          wd[r] = ok ? __float_as_uint(dd) : kCgNone;
        }
        const uint32_t m = min(min(wd[0], wd[1]), min(wd[2], wd[3]));
        const uint64_t e = ((uint64_t)m << 32) | ((uint64_t)(uint32_t)(base + row0) << 4);
        // (lanes past the last frame keep nothing: their slots are another's)
        if (fr[j] < a.nq && m != kCgNone && e < lst[j][kCgKeep - 1]) {
          const int slot = (int)(lst[j][kCgKeep - 1] & 15);
          cg_insert(lst[j], e | (uint64_t)slot);
          reinterpret_cast<v4u *>(a.slots)[slot_base[j] + slot] = v4u{wd[0], wd[1], wd[2], wd[3]};
        }
      }
    }
    HLOC_CG_STAGE(buf ^ 1)  // last read before the previous barrier
    __syncthreads();
    cur_t = advance(cur_t);
  }
#undef HLOC_CG_FETCH
#undef HLOC_CG_STAGE
  // per (frame, split, lane group): 4 keys per kept quad and the bound
#pragma unroll
  for (int j = 0; j < 2; ++j) {
    if (fr[j] >= a.nq) continue;
    const int64_t lidx = ((int64_t)fr[j] * a.splits + split) * 4 + g;
    uint64_t *out = a.keys + lidx * (kCgKeep * 4);
#pragma unroll
    for (int e = 0; e < kCgKeep; ++e) {
      const uint64_t ent = lst[j][e];
      const uint32_t m = (uint32_t)(ent >> 32);
      v4u wq = v4u{kCgNone, kCgNone, kCgNone, kCgNone};
      if (m != kCgNone) wq = reinterpret_cast<const v4u *>(a.slots)[slot_base[j] + (int)(ent & 15)];
      const uint32_t q0 = (uint32_t)(ent >> 4) & 0x0FFFFFFFu;
      const uint32_t ww[4] = {wq.x, wq.y, wq.z, wq.w};
#pragma unroll
      for (int r = 0; r < 4; ++r)
        out[e * 4 + r] = ww[r] == kCgNone ? kKeyNone : (((uint64_t)ww[r] << 32) | (q0 + r));
    }
    const uint32_t lm = (uint32_t)(lst[j][kCgKeep - 1] >> 32);
    a.bounds[lidx] = lm == kCgNone ? kKeyNone : ((uint64_t)lm << 32);
  }
}

template <int NS>
constexpr size_t coarse_gemm_lds() {
  return (size_t)2 * kCgTile * (4 * NS + 1) * sizeof(v4u);
}

bool coarse_gemm_supports(int32_t dp) {
  const int ns = dp / 32;
  return dp % 64 == 0 && ns >= 2 && ns <= 16;
}

// Splits of the representatives: enough blocks to give every compute unit
// two, each split at least 64 representatives.
int32_t coarse_gemm_splits(int32_t nq, int32_t R, int32_t num_cu) {
  const int64_t tiles = std::max<int64_t>(1, (nq + kCgFrames - 1) / kCgFrames);
  int64_t s = (2 * (int64_t)num_cu + tiles - 1) / tiles;
  s = std::min<int64_t>(s, std::max<int64_t>(1, R / 64));
  return (int32_t)std::max<int64_t>(1, std::min<int64_t>(s, 64));
}

template <int NS>
hipError_t launch_cg_ns(CoarseGemmArgs a, hipStream_t s) {
  const int64_t tiles = (a.nq + kCgFrames - 1) / kCgFrames;
  const dim3 grid((unsigned)(tiles * a.splits));
  const uint32_t lds = (uint32_t)coarse_gemm_lds<NS>();
  return a.rlabel ? launch_kernel(k_coarse_gemm<NS, true>, grid, dim3(256), lds, s, a)
                  : launch_kernel(k_coarse_gemm<NS, false>, grid, dim3(256), lds, s, a);
}

hipError_t launch_coarse_gemm(CoarseGemmArgs a, hipStream_t s) {
  if (a.nq <= 0) return hipSuccess;
  if (!coarse_gemm_supports(a.dp) || a.splits < 1 || a.reps_per_split < 1 ||
      (int64_t)a.splits * a.reps_per_split < a.R ||
      (int64_t)a.nq * a.splits * 4 * kCgKeep >= ((int64_t)1 << 31))
    return hipErrorInvalidValue;
  switch (a.dp / 32) {
    case 2: return launch_cg_ns<2>(a, s);
    case 4: return launch_cg_ns<4>(a, s);
    case 6: return launch_cg_ns<6>(a, s);
    case 8: return launch_cg_ns<8>(a, s);
    case 10: return launch_cg_ns<10>(a, s);
    case 12: return launch_cg_ns<12>(a, s);
    case 14: return launch_cg_ns<14>(a, s);
    case 16: return launch_cg_ns<16>(a, s);
    default: return hipErrorInvalidValue;
  }
}

hipError_t prepare_coarse_gemm_kernels() {
#define HLOC_CG_ATTR(N)                                                                    \
  for (const void *k : {reinterpret_cast<const void *>(&k_coarse_gemm<N, false>),          \
                        reinterpret_cast<const void *>(&k_coarse_gemm<N, true>)}) {        \
    const hipError_t e = hipFuncSetAttribute(k, hipFuncAttributeMaxDynamicSharedMemorySize, \
                                             (int)coarse_gemm_lds<N>());                    \
    if (e != hipSuccess) return e;                                                         \
  }
  HLOC_CG_ATTR(2)
  HLOC_CG_ATTR(4)
  HLOC_CG_ATTR(6)
  HLOC_CG_ATTR(8)
  HLOC_CG_ATTR(10)
  HLOC_CG_ATTR(12)
  HLOC_CG_ATTR(14)
  HLOC_CG_ATTR(16)
#undef HLOC_CG_ATTR
  return hipSuccess;
}

}  // namespace hloc
