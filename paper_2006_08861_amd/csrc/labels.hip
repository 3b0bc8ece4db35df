// Subspace labels (Section 4 keeps the top N candidates of every walked path:
// N x M x P of them for a request of M frames over P paths). A query over
// labels runs the two-stage search once per label with the coarse words of
// every region outside the label set to "no candidate", so that the coarse
// selection, the fine screen and the top-k stay within the label; the
// aggregation then pools, for each frame of a request, the k results of
// every label.
#include <algorithm>

#include "hloc_host.h"

namespace hloc {

// words: nq x R coarse screen words (frame-major); those of regions whose
// label is not the frame's become 0xFFFFFFFF (no candidate). The frame's
// label is p, or, with per > 0, frame / per (a batch holding the frames once
// per label).
__global__ void k_mask_label(uint32_t *words, int64_t total, int R,
                             const int32_t *__restrict__ rlabel, int p, int per) {
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < total;
       i += (int64_t)gridDim.x * blockDim.x) {
    const int lab = per > 0 ? (int)((i / R) / per) : p;
    if (rlabel[i % R] != lab) words[i] = 0xFFFFFFFFu;
  }
}

hipError_t launch_mask_label(uint32_t *words, int32_t nq, int32_t R, const int32_t *rlabel,
                             int32_t p, int32_t per, hipStream_t s) {
  const int64_t total = (int64_t)nq * R;
  if (total <= 0) return hipSuccess;
  const int grid = (int)std::min<int64_t>((total + 255) / 256, 8192);
  return launch_kernel(k_mask_label, dim3(grid), dim3(256), 0, s, words, total, R, rlabel, p,
                       per);
}

// Frame lists of the labelled query: the results of frame f under label p
// are row p * nq + f of the stacked per-label lists; request r pools the
// entries P * off[r] .. P * off[r+1] - 1, entry P * f + p naming that row.
__global__ void k_label_lists(const int32_t *__restrict__ req_offsets, int nreq, int nq, int P,
                              int32_t *list_off, int32_t *list) {
  const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (t <= nreq) list_off[t] = P * (req_offsets ? req_offsets[t] : (int32_t)t);
  if (t < (int64_t)nq * P) {
    const int f = (int)(t / P), p = (int)(t % P);
    list[t] = p * nq + f;
  }
}

hipError_t launch_label_lists(const int32_t *req_offsets, int32_t nreq, int32_t nq, int32_t P,
                              int32_t *list_off, int32_t *list, hipStream_t s) {
  const int64_t n = std::max<int64_t>((int64_t)nq * P, (int64_t)nreq + 1);
  return launch_kernel(k_label_lists, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, s,
                       req_offsets, nreq, nq, P, list_off, list);
}

}  // namespace hloc
