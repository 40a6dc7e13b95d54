// The Galerkin product by aggregate index (Section 3.1, eq. galerkin) for a
// given aggregation, without any allocation: amg_galerkin's kernels (input
// checks, aggregate segments, staged terms, wave-hash reduce, compaction)
// with all their scratch in one static device array of fixed size, for
// callers that cannot allocate device or pinned memory.
//
// The array is a device symbol: host code never passes its name to a kernel
// (on the host that name is only a stand-in, not a device address).  The
// first call on a device, with that device current, takes the array's
// device address with hipGetSymbolAddress and keeps it for that device; every
// launch and fill uses that address.  Every call on one device shares the
// array: the parts that must start at zero are cleared at the start of each
// call, and calls that overlap on one device (two streams, two threads) race.
#include <hip/hip_runtime.h>

#include <mutex>
#include <string>

#include "amg_internal.hpp"

namespace amg {
namespace {

constexpr int kNaMaxRows = 1 << 17;    // n <= 131,072 fine rows
constexpr int kNaMaxNnz = 1 << 20;     // nnz <= 1,048,576 stored entries
constexpr int kNaMaxDevices = 64;

constexpr size_t align256(size_t b) { return (b + 255) / 256 * 256; }

// Byte offsets inside the scratch array.
constexpr size_t kOffTkey = 0;                                                    // int[nnz]
constexpr size_t kOffTval = kOffTkey + align256(sizeof(int) * kNaMaxNnz);         // double[nnz]
constexpr size_t kOffLens = kOffTval + align256(sizeof(double) * kNaMaxNnz);      // int[n]
constexpr size_t kOffToff = kOffLens + align256(sizeof(int) * kNaMaxRows);        // int[n + 1]
constexpr size_t kOffAggPtr = kOffToff + align256(sizeof(int) * (kNaMaxRows + 1));   // int[nc + 1]
constexpr size_t kOffAggRows = kOffAggPtr + align256(sizeof(int) * (kNaMaxRows + 1));  // int[n]
constexpr size_t kOffCounts = kOffAggRows + align256(sizeof(int) * kNaMaxRows);   // int[nc]
constexpr size_t kOffUcount = kOffCounts + align256(sizeof(int) * kNaMaxRows);    // int[nc]
constexpr size_t kOffList = kOffUcount + align256(sizeof(int) * kNaMaxRows);      // int[2 nc]
constexpr size_t kOffCtl = kOffList + align256(sizeof(int) * 2 * (size_t)kNaMaxRows);   // int[64]: 0-1 tier
                                                                                        // counters, 32 error bits
constexpr int kScanBlocks = (kNaMaxRows + 4095) / 4096;   // tiles of 4096 in the longest scan
constexpr size_t kOffScan = kOffCtl + align256(sizeof(int) * 64);                 // uint64[tiles + 1]: look-back
                                                                                  // words, then the ticket
constexpr size_t kNaBytes = kOffScan + align256(sizeof(uint64_t) * (kScanBlocks + 1));

static __device__ __align__(256) unsigned char scratch[kNaBytes];

struct DeviceScratch {
  bool ready = false;
  unsigned char* ptr = nullptr;   // device address of `scratch` on this device
  ScanCtx scan;                   // look-back words inside the array, epoch kept across calls
};
std::mutex g_na_mu;
DeviceScratch g_na[kNaMaxDevices];

// Device address of the array on the current device (taken once per device).
DeviceScratch& device_scratch() {
  int dev = 0;
  AMG_HIP(hipGetDevice(&dev));
  if (dev < 0 || dev >= kNaMaxDevices) throw Error(AMG_EUNSUPPORTED, "device index beyond the scratch table");
  std::lock_guard<std::mutex> g(g_na_mu);
  DeviceScratch& d = g_na[dev];
  if (!d.ready) {
    void* p = nullptr;
    AMG_HIP(hipGetSymbolAddress(&p, HIP_SYMBOL(scratch)));
    if (!p) throw Error(AMG_EHIP, "hipGetSymbolAddress returned no address for the scratch array");
    d.ptr = static_cast<unsigned char*>(p);
    d.scan.status = reinterpret_cast<uint64_t*>(d.ptr + kOffScan);
    d.scan.ticket = reinterpret_cast<unsigned long long*>(d.scan.status + kScanBlocks);
    d.scan.max_blocks = kScanBlocks;
    d.scan.epoch = 1;
    d.ready = true;
  }
  return d;
}

template <typename T>
T* at(unsigned char* base, size_t off) { return reinterpret_cast<T*>(base + off); }

// Waits for the stream and turns the device error word into a status.
void wait_and_check(const int* d_err, hipStream_t s) {
  AMG_HIP(hipGetLastError());
  int e = 0;
  AMG_HIP(hipMemcpyAsync(&e, d_err, sizeof(int), hipMemcpyDeviceToHost, s));
  AMG_HIP(hipStreamSynchronize(s));
  if (!e) return;
  if (e & kErrNonFinite) throw Error(AMG_ENANINF, "non-finite matrix entry");
  if (e & kErrZeroDiag) throw Error(AMG_EINVAL, "zero or missing diagonal entry");
  if (e & kErrBadColumn) throw Error(AMG_EINVAL, "column or aggregate index out of range, or columns not increasing");
  if (e & kErrNonSymPattern) throw Error(AMG_EINVAL, "sparsity pattern is not structurally symmetric");
  throw Error(AMG_EHIP, "device error bits " + std::to_string(e));
}

}  // namespace

int galerkin_noalloc(const amg_csr& A, const int* agg, const double* pval, int nc, int* row_ptr_c, int* col_c,
                     double* val_c, int cap, int* nnz_c, hipStream_t s) {
  if (A.n > kNaMaxRows || A.nnz > kNaMaxNnz)
    throw Error(AMG_EINVAL, "matrix larger than the scratch array (n <= " + std::to_string(kNaMaxRows) +
                                ", nnz <= " + std::to_string(kNaMaxNnz) + ")");
  DeviceScratch& d = device_scratch();
  unsigned char* base = d.ptr;
  const int n = A.n, nnz = A.nnz;
  int* ctl = at<int>(base, kOffCtl);
  int* err = ctl + 32;
  // what must start at zero: tier counters, error word, look-back words and
  // the scan ticket (a call cut short by an error can leave them set)
  launch_fill_int(64, ctl, 0, s);
  launch_fill_int(2 * ((size_t)kScanBlocks + 1), reinterpret_cast<int*>(d.scan.status), 0, s);
  d.scan.epoch = 1;

  // row pointers bracket the stored entries; then the per-entry checks
  int ends[2] = {-1, -1};
  AMG_HIP(hipMemcpyAsync(&ends[0], A.row_ptr, sizeof(int), hipMemcpyDeviceToHost, s));
  AMG_HIP(hipMemcpyAsync(&ends[1], A.row_ptr + n, sizeof(int), hipMemcpyDeviceToHost, s));
  AMG_HIP(hipStreamSynchronize(s));
  if (ends[0] != 0 || ends[1] != nnz) throw Error(AMG_EINVAL, "row_ptr[0] != 0 or row_ptr[n] != nnz");
  launch_check_rowptr(n, A.row_ptr, err, s);
  wait_and_check(err, s);
  launch_check_matrix(n, A.row_ptr, A.col_idx, A.val, err, s);
  launch_check_index(n, agg, nc, err, s);
  wait_and_check(err, s);

  // aggregate segments: members of aggregate I ascending at
  // agg_rows[agg_ptr[I] .. agg_ptr[I+1])
  int* agg_ptr = at<int>(base, kOffAggPtr);
  int* agg_rows = at<int>(base, kOffAggRows);
  int* counts = at<int>(base, kOffCounts);
  launch_fill_int(nc, counts, 0, s);
  launch_agg_count(n, agg, counts, s);
  scan_to_ptr(counts, agg_ptr, nc, d.scan, s);
  launch_fill_int(nc, counts, 0, s);
  launch_agg_scatter(n, agg, agg_ptr, counts, agg_rows, s);
  launch_agg_sort(nc, agg_ptr, agg_rows, s);

  // terms in segment order, reduced per coarse row; row pointers of A_c
  GalerkinScratch g;
  g.lens = at<int>(base, kOffLens);
  g.toff = at<int>(base, kOffToff);
  g.tkey = at<int>(base, kOffTkey);
  g.tval = at<double>(base, kOffTval);
  g.ucount = at<int>(base, kOffUcount);
  g.list = at<int>(base, kOffList);
  g.ctl = ctl;
  launch_galerkin_stage(g, n, nc, nnz, A.row_ptr, A.col_idx, A.val, agg, pval, agg_ptr, agg_rows, d.scan, s);
  scan_to_ptr(g.ucount, row_ptr_c, nc, d.scan, s);
  int total = 0;
  AMG_HIP(hipMemcpyAsync(&total, row_ptr_c + nc, sizeof(int), hipMemcpyDeviceToHost, s));
  wait_and_check(err, s);
  *nnz_c = total;
  if (total > cap) return AMG_EINVAL;
  launch_galerkin_finish(g, nc, agg_ptr, row_ptr_c, col_c, val_c, s);
  wait_and_check(err, s);
  return AMG_OK;
}

}  // namespace amg
