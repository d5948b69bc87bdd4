// ct_split.hip -- device halves of the split propagators (include/ct.h,
// ct_split_*): the two variants of Sec. 4 that run only one of the two CT
// procedures on the device.
//
//   update variant (Sec. 4.1): the device computes updateTable's mask
//     (Alg. 2): for every changed variable, the OR of the support rows it
//     names, complemented on the incremental branch, and the AND of those
//     per-variable masks; the host ANDs it into its currTable.
//   filter variant (Sec. 4.2): the device runs filterDomains (Alg. 3) over
//     the domain words of the variables in s_sup, against a currTable that
//     the host updated and sent along with the domains.
//
// Both are plain bitwise streams over support rows, coalesced along the
// currTable words; neither keeps any CT state on the device beyond the
// residues of the filter variant (hints only: any word index is a valid
// residue, so they need no restoring on backtrack).
#include <hip/hip_runtime.h>

#include <cstdint>

#include "ct_device.h"

namespace ctk {
namespace {

constexpr int SPLIT_BLOCK = 256;
constexpr int SPLIT_WAVES = SPLIT_BLOCK / WAVE;

// One thread per currTable word: mask[w] = AND over the segments of
// (OR of the segment's rows at word w), complemented for incremental
// segments.  Segment s covers rowList[segBegin[s] .. segBegin[s + 1]); a
// negative segBegin entry marks an incremental segment (the begin is then
// -1 - begin).  The mask goes straight to host memory; each workgroup then
// publishes `seq` in its flag, after a system-scope fence, so the host
// knows its part has landed.
__global__ __launch_bounds__(SPLIT_BLOCK) void split_update_kernel(
    const uint64_t* __restrict__ S, int64_t stride, int64_t W, const int32_t* __restrict__ segBegin,
    int nSeg, const int32_t* __restrict__ rowList, uint64_t* __restrict__ mask, int32_t* flags, int32_t seq) {
  const int64_t w = (int64_t)blockIdx.x * SPLIT_BLOCK + threadIdx.x;
  if (w < W) {
    uint64_t acc = ~0ull;
    for (int s = 0; s < nSeg; ++s) {
      const int32_t b0 = segBegin[s], b1 = segBegin[s + 1];
      const bool inc = b0 < 0;
      const int begin = inc ? -1 - b0 : b0;
      const int end = b1 < 0 ? -1 - b1 : b1;
      uint64_t m = 0;
      for (int k = begin; k < end; ++k) m |= S[(int64_t)rowList[k] * stride + w];
      acc &= inc ? ~m : m;
    }
    mask[w] = acc;
  }
  __threadfence_system();
  __syncthreads();
  if (threadIdx.x == 0) __hip_atomic_store(&flags[blockIdx.x], seq, __ATOMIC_RELEASE, __HIP_MEMORY_SCOPE_SYSTEM);
}

// One wave per listed domain word, one value per lane.  A present value
// stays if its support row meets currTable at its residue word; otherwise
// the wave scans currTable 64 words at a time for the first word where they
// meet (the new residue), and the value is removed if there is none.
// wordRow[k] is the support row of bit 0 of domain word k.  The host has
// checked that no bit past a variable's domain size is set, so every
// present lane names a row of the table.  The filtered word goes straight
// to host memory (domOut[k]); each workgroup then publishes `seq` in its
// flag, after a system-scope fence.
__global__ __launch_bounds__(SPLIT_BLOCK) void split_filter_kernel(
    const uint64_t* __restrict__ S, int64_t stride, int64_t W, const uint64_t* __restrict__ ct,
    const uint64_t* __restrict__ dom, const int32_t* __restrict__ words, int nWords,
    const int32_t* __restrict__ wordRow, int32_t* __restrict__ res, uint64_t* __restrict__ domOut,
    int32_t* flags, int32_t seq) {
  const int item = blockIdx.x * SPLIT_WAVES + (int)(threadIdx.x / WAVE);
  const int lane = threadIdx.x & (WAVE - 1);
  if (item < nWords) {  // wave-uniform
    const int k = words[item];
    const uint64_t d = dom[k];
    const int row = wordRow[k] + lane;
    const bool present = (d >> lane) & 1ull;
    bool keep = false;
    if (present) {
      const int r = res[row];
      keep = (ct[r] & S[(int64_t)row * stride + r]) != 0;
    }
    uint64_t missing = __ballot(present && !keep);
    while (missing) {
      const int l = __ffsll((unsigned long long)missing) - 1;
      missing &= missing - 1;
      const int64_t rowOff = (int64_t)(wordRow[k] + l) * stride;
      int64_t found = -1;
      for (int64_t base = 0; base < W; base += WAVE) {
        const int64_t w = base + lane;
        bool hit = false;
        if (w < W) hit = (ct[w] & S[rowOff + w]) != 0;
        const uint64_t b = __ballot(hit);
        if (b) {
          found = base + __ffsll((unsigned long long)b) - 1;
          break;
        }
      }
      if (lane == l && found >= 0) {
        res[row] = (int32_t)found;
        keep = true;
      }
    }
    const uint64_t kept = __ballot(keep);
    if (lane == 0) domOut[k] = kept;
  }
  __threadfence_system();
  __syncthreads();
  if (threadIdx.x == 0) __hip_atomic_store(&flags[blockIdx.x], seq, __ATOMIC_RELEASE, __HIP_MEMORY_SCOPE_SYSTEM);
}

}  // namespace

int split_update_grid(int64_t W) { return (int)((W + SPLIT_BLOCK - 1) / SPLIT_BLOCK); }
int split_filter_grid(int nWords) { return (nWords + SPLIT_WAVES - 1) / SPLIT_WAVES; }

// `grid` flags receive `seq` (one per workgroup) once that workgroup's
// outputs are visible to the host.
hipError_t launch_split_update(const uint64_t* S, int64_t stride, int64_t W, const int32_t* segBegin,
                               int nSeg, const int32_t* rowList, uint64_t* mask, int32_t* flags, int32_t seq,
                               hipStream_t stream) {
  if (W <= 0) return hipSuccess;
  hipLaunchKernelGGL(split_update_kernel, dim3((unsigned)split_update_grid(W)), dim3(SPLIT_BLOCK), 0, stream, S,
                     stride, W, segBegin, nSeg, rowList, mask, flags, seq);
  return hipGetLastError();
}

hipError_t launch_split_filter(const uint64_t* S, int64_t stride, int64_t W, const uint64_t* ct,
                               const uint64_t* dom, const int32_t* words, int nWords, const int32_t* wordRow,
                               int32_t* res, uint64_t* domOut, int32_t* flags, int32_t seq, hipStream_t stream) {
  if (W <= 0 || nWords <= 0) return hipSuccess;
  hipLaunchKernelGGL(split_filter_kernel, dim3(split_filter_grid(nWords)), dim3(SPLIT_BLOCK), 0, stream, S,
                     stride, W, ct, dom, words, nWords, wordRow, res, domOut, flags, seq);
  return hipGetLastError();
}

}  // namespace ctk
