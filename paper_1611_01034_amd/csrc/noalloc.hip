// ddamg_apply_dirac_noalloc: the fine operator D(+-mu) = D_W +- i Gamma5 mu
// (Sec. 1) on device fields, for callers that cannot allocate device memory.
// It runs the kernels of ddamg_apply_dirac in FP64 (lexicographic -> block
// layout, D, block layout -> lexicographic); the two block-layout fields live
// in the file-scope array below instead of the context's buffers.
#include <mutex>

#include "solver.hpp"

struct ddamg_ctx {
  ddamg::Ctx c;
};

namespace ddamg {

// Largest lattice the scratch serves: 131072 sites (16^3 x 32).  Two FP64
// spinor fields in block layout, 2 * 131072 * 12 * 16 bytes = 48 MiB, held by
// every device the library runs on until the process ends.  Host code never
// passes the array's name to a kernel or a copy: it uses the address that
// hipGetSymbolAddress returns on each device.
constexpr long kNoAllocMaxSites = 131072;
constexpr size_t kScratchBytes = 2 * (size_t)kNoAllocMaxSites * 12 * sizeof(cx<double>);
static __device__ __align__(256) unsigned char scratch[kScratchBytes];

namespace {
constexpr int kMaxDevices = 64;
std::mutex g_mu;
void* g_scratch[kMaxDevices] = {};
}  // namespace

// Called by ddamg_create with the context's device current: records that
// device's address of the scratch array (once per device).
void noalloc_scratch_init(int dev) {
  if (dev < 0 || dev >= kMaxDevices) throw Error(INVALID_ARG, "device index out of range");
  std::lock_guard<std::mutex> lk(g_mu);
  if (g_scratch[dev]) return;
  void* p = nullptr;
  HIP_CHECK(hipGetSymbolAddress(&p, HIP_SYMBOL(scratch)));
  if (!p) throw Error(HIP_FAIL, "no device address for the scratch array");
  g_scratch[dev] = p;
}

static void* scratch_of(int dev) {
  if (dev < 0 || dev >= kMaxDevices) return nullptr;
  std::lock_guard<std::mutex> lk(g_mu);
  return g_scratch[dev];
}

}  // namespace ddamg

using namespace ddamg;

extern "C" int ddamg_apply_dirac_noalloc(ddamg_ctx* ctx, const void* in, void* out, int sign) {
  if (!ctx) return DDAMG_INVALID_ARG;
  Ctx& c = ctx->c;
  try {
    c.err.clear();
    if (!c.have_gauge) throw Error(BAD_STATE, "no gauge field set");
    if (!in || !out) throw Error(INVALID_ARG, "NULL field");
    if (sign != 1 && sign != -1) throw Error(INVALID_ARG, "sign must be +1 or -1");
    if (c.g.V > kNoAllocMaxSites)
      throw Error(INVALID_ARG, "lattice of " + std::to_string(c.g.V) +
                                   " sites exceeds the no-allocation scratch (at most 131072 sites)");
    cx<double>* a = (cx<double>*)scratch_of(c.dev);
    if (!a) throw Error(BAD_STATE, "scratch array not set up on the context's device");
    cx<double>* b = a + kNoAllocMaxSites * 12;
    // every entry of the first V*12 of each half is written before it is read
    launch_from_lex<double>(c.g, (const cx<double>*)in, a, 12, c.st);
    launch_dirac<double, double>(c.g, c.U64.p, c.H64.as<double>(), c.twist(sign), a, b, c.st);
    launch_to_lex<double>(c.g, b, (cx<double>*)out, 12, c.st);
    HIP_CHECK(hipGetLastError());
    return DDAMG_OK;
  } catch (const Error& e) {
    c.err = e.what();
    return e.status;
  } catch (const HipError& e) {
    c.err = e.what();
    return DDAMG_HIP_ERROR;
  } catch (const std::exception& e) {
    c.err = e.what();
    return DDAMG_HIP_ERROR;
  }
}
