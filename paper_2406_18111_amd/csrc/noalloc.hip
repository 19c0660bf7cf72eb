// Single-window analysis that allocates nothing during the call: its
// workspace is a fixed device array of this file (one copy per GPU, held
// until the process ends), laid out once per device when a context is
// created on it.  For callers that cannot allocate device memory while they
// run (tight serving loops, harnesses that forbid allocation).
#include "apo.h"
#include "pipeline.h"
#include "stages.h"
#include <cstdio>
#include <mutex>

namespace apo {

constexpr int kNoAllocDevices = 64;

// The workspace of one analysis of up to APO_NOALLOC_MAX_N tokens.  In host
// code this name is only a stand-in for the symbol: the device address comes
// from hipGetSymbolAddress, per device.
static __device__ __align__(256) uint8_t scratch[APO_NOALLOC_SCRATCH_BYTES];

struct NoAllocDevice {
  std::once_flag once;
  int rc = APO_EDEVICE;     // outcome of the set-up on this device
  void *ptr = nullptr;      // this device's copy of `scratch`
  Workspace ws;             // laid out over ptr
  std::mutex mu;            // one analysis at a time per device
};
static NoAllocDevice g_noalloc[kNoAllocDevices];

// Once per device, with that device current (called from apo_create).
int noalloc_setup(int device) {
  if (device < 0 || device >= kNoAllocDevices) return APO_EINVAL;
  NoAllocDevice &D = g_noalloc[device];
  std::call_once(D.once, [&D] {
    void *p = nullptr;
    const hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
    if (e != hipSuccess || !p) {
      fprintf(stderr, "[apo] no-allocation scratch: hipGetSymbolAddress failed: %s\n", hipGetErrorString(e));
      (void)hipGetLastError();
      D.rc = APO_EDEVICE;
      return;
    }
    D.ptr = p;
    const int rc = D.ws.attach(p, APO_NOALLOC_SCRATCH_BYTES, APO_NOALLOC_MAX_N, 1);
    if (rc) {
      fprintf(stderr, "[apo] no-allocation scratch: workspace of %llu tokens does not fit %llu bytes\n",
              (unsigned long long)APO_NOALLOC_MAX_N, (unsigned long long)APO_NOALLOC_SCRATCH_BYTES);
      D.ws.release();
      D.rc = rc == -2 ? APO_ENOMEM : APO_EDEVICE;
      return;
    }
    D.rc = APO_OK;
  });
  return D.rc;
}

int noalloc_run(int device, hipStream_t s, int tile_log, int digit_bits, const void *d_tok, int bits, uint32_t n,
                uint32_t min_len, apo_candidate *d_out, uint32_t out_cap, uint32_t *h_out_n, apo_occurrence *d_occ,
                uint32_t occ_cap, uint32_t *h_occ_n, RunInfo &info) {
  if (device < 0 || device >= kNoAllocDevices) return APO_EINVAL;
  NoAllocDevice &D = g_noalloc[device];
  if (D.rc != APO_OK) return D.rc;
  if (n > APO_NOALLOC_MAX_N) return APO_ENOMEM;
  std::lock_guard<std::mutex> lk(D.mu);
  Workspace &w = D.ws;
  // The array keeps the previous call's contents: clear what the stages
  // expect to find zeroed (device counters, the sort engine's histograms and
  // counters), with fill kernels.
  SortBufs &B = w.eng.bufs();
  fill_u32(w.dcnt, CNT_COUNT, 0, s);
  fill_u32(B.hist, (uint64_t)B.big_cap * kBins, 0, s);
  fill_u32(reinterpret_cast<uint32_t *>(B.ctr), sizeof(SortCounters) / 4, 0, s);
  w.sel_cap = kSelRoundCap;
  w.sel_prefix = -1;
  w.win_greedy = true;
  w.fail_after = -1;
  w.ktag = KT_NONE;
  w.eng.set_params(tile_log, digit_bits);
  const uint64_t off[2] = {0, n};
  int rc = run_pipeline(w, d_tok, bits, n, off, 1, min_len, Stop::FULL, s, info, Mode::HOST);
  if (rc) return rc == -2 ? APO_ENOMEM : APO_EDEVICE;
  const uint32_t rows = info.rows, acc = info.accepted;
  *h_out_n = rows;
  if (h_occ_n) *h_occ_n = acc;
  if (rows > out_cap || (d_occ && acc > occ_cap)) return APO_ERANGE;
  if (rows && hipMemcpyAsync(d_out, w.rows, (size_t)rows * sizeof(apo_candidate), hipMemcpyDeviceToDevice, s) !=
                  hipSuccess)
    return APO_EDEVICE;
  if (d_occ && acc &&
      hipMemcpyAsync(d_occ, w.occ, (size_t)acc * sizeof(apo_occurrence), hipMemcpyDeviceToDevice, s) != hipSuccess)
    return APO_EDEVICE;
  return hipStreamSynchronize(s) == hipSuccess ? APO_OK : APO_EDEVICE;
}

}  // namespace apo
