// Allocation-free projected Gauss-Seidel (icr_solve_contacts_noalloc): the
// same kernels as icr_solve_contacts, with every work buffer carved out of
// one file-scope device array instead of a scene's arena.  For callers that
// cannot allocate device memory (code under HIP graph capture, tight serving
// loops, harnesses that forbid hipMalloc).
//
// The array's name is a host-side stand-in in host code: its device address
// is looked up once per device (hipGetSymbolAddress, with that device
// current) and only that address is handed to kernels.  Every call on a
// device shares that device's copy, so calls that overlap on one GPU race.
// Nothing in it has to start at zero: within a call, each kernel writes the
// part of the array that a later kernel reads (start gaps, first active set,
// its records and coupling blocks, the control words, sweeps and eps).  A
// set that outgrows the register chains continues in the block Gauss-Seidel
// over the whole GPU, whose buffers are part of the array too (under stream
// capture, in the single-workgroup sweep).
#include <mutex>

#include "scene.hpp"

namespace icr {

namespace {

constexpr int kNoAllocMaxContacts = 1024;
constexpr int kMaxDevices = 64;

// Layout in doubles; every region starts on a 256-byte boundary.
constexpr size_t align32(size_t n) { return (n + 31) / 32 * 32; }
constexpr size_t kOffG = 0;                                                        // g [3 nc]
constexpr size_t kOffWss = kOffG + align32(3 * kNoAllocMaxContacts);               // blocked W~_SS
constexpr size_t kOffGnSet = kOffWss + align32(pgs_wss_elems(kNoAllocMaxContacts));
constexpr size_t kOffSwn = kOffGnSet + align32(kNoAllocMaxContacts);
constexpr size_t kOffRec = kOffSwn + align32(kNoAllocMaxContacts);
constexpr size_t kOffGS = kOffRec + align32(pgs_rec_elems(kNoAllocMaxContacts));
constexpr size_t kOffEps = kOffGS + align32(pgs_rec_elems(kNoAllocMaxContacts));   // eps [1]
// block Gauss-Seidel of sets beyond the register chains
constexpr size_t kOffRecAll = kOffEps + 32;                                         // records of all contacts
constexpr size_t kOffWblk = kOffRecAll + align32((size_t)kNoAllocMaxContacts * kPgsRecWidth);
constexpr size_t kOffDl = kOffWblk + align32(pgs_coop_blk_elems(kNoAllocMaxContacts));
constexpr size_t kOffInts = kOffDl + align32(2 * 3 * kPgsCoopB);                   // ints below
constexpr size_t kIntSidx = 0, kIntNS = kNoAllocMaxContacts, kIntCtl = kIntNS + 1, kIntSweeps = kIntCtl + 4,
                 kIntChg = kIntSweeps + 1, kIntSync = kIntChg + 2 * kPgsCoopB;
constexpr size_t kInts = kIntSync + kPgsCoopSync;
constexpr size_t kScratchDoubles = kOffInts + align32((kInts + 1) / 2);

// About 32 MB per GPU, held until the process ends.
__device__ __align__(256) double scratch[kScratchDoubles];

std::mutex g_mtx;
double *g_ptr[kMaxDevices] = {};

// Device address of this device's copy of `scratch` (looked up on the first
// call on the device).
double *scratch_ptr() {
  int dev = 0;
  ICR_HIP(hipGetDevice(&dev));
  if (dev < 0 || dev >= kMaxDevices) throw std::runtime_error("device ordinal beyond the scratch table");
  std::lock_guard<std::mutex> lock(g_mtx);
  if (!g_ptr[dev]) {
    void *p = nullptr;
    ICR_HIP(hipGetSymbolAddress(&p, HIP_SYMBOL(scratch)));
    if (!p) throw std::runtime_error("hipGetSymbolAddress returned NULL");
    g_ptr[dev] = static_cast<double *>(p);
  }
  return g_ptr[dev];
}

}  // namespace

}  // namespace icr

extern "C" icr_status icr_solve_contacts_noalloc(void *stream, int32_t n_c, const double *W, const double *d,
                                                 const double *mu, double h, double *lambda, int8_t *status,
                                                 int32_t max_sweeps, double tol, int32_t j_inner,
                                                 int32_t *sweeps_out, double *eps_out) {
  using namespace icr;
  if (n_c < 1 || n_c > kNoAllocMaxContacts) return ICR_E_ARG;
  if (max_sweeps < 1 || j_inner < 0 || !std::isfinite(h) || !(h > 0)) return ICR_E_ARG;
  if (!W || !d || !mu || !lambda || !status) return ICR_E_ARG;
  try {
    hipStream_t st = (hipStream_t)stream;
    double *base = scratch_ptr();
    int *ints = reinterpret_cast<int *>(base + kOffInts);
    PgsWork wk;
    wk.g = base + kOffG;
    wk.Wss = base + kOffWss;
    wk.gnSet = base + kOffGnSet;
    wk.swn = base + kOffSwn;
    wk.rec = base + kOffRec;
    wk.gS = base + kOffGS;
    wk.Sidx = ints + kIntSidx;
    wk.nS = ints + kIntNS;
    wk.ctl = ints + kIntCtl;
    wk.recAll = base + kOffRecAll;
    wk.Wblk = base + kOffWblk;
    wk.dl = base + kOffDl;
    wk.chg = ints + kIntChg;
    wk.csync = ints + kIntSync;
    int *sweeps_dev = ints + kIntSweeps;
    double *eps_dev = base + kOffEps;
    pgs_prepare();
    launch_pgs<double>(st, n_c, W, d, mu, h, lambda, status, max_sweeps, tol, j_inner, sweeps_dev, eps_dev, wk);
    if (sweeps_out || eps_out) {
      int sw = 0;
      double ep = 0;
      ICR_HIP(hipMemcpyAsync(&sw, sweeps_dev, sizeof(int), hipMemcpyDeviceToHost, st));
      ICR_HIP(hipMemcpyAsync(&ep, eps_dev, sizeof(double), hipMemcpyDeviceToHost, st));
      ICR_HIP(hipStreamSynchronize(st));
      if (sweeps_out) *sweeps_out = sw;
      if (eps_out) *eps_out = ep;
      if (!(ep <= tol)) return ICR_WARN_NOT_CONVERGED;
    }
    return ICR_OK;
  } catch (const HipError &) {
    return ICR_E_HIP;
  } catch (...) {
    return ICR_E_HIP;
  }
}
