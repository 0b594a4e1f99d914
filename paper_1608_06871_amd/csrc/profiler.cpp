// Optional per-launch timing of the library's kernels with HIP events on the
// launch stream, accumulated per kernel class with the launch's algorithmic
// flops and bytes.  Disabled unless hps_profile_start() was called.
#include <atomic>
#include <cstring>
#include <mutex>
#include <vector>

#include "../../include/hps_blocks.h"
#include "common.h"

namespace hps {
namespace {

struct Rec {
  hipEvent_t a, b;
  int kind, phase;
  double flops, bytes;
};

std::atomic<bool> g_on{false};
std::atomic<int> g_phase{0};
const char* const PHASE_NAMES[PHASE_COUNT] = {"phase:other", "phase:leaf", "phase:merge", "phase:top",
                                              "phase:solve", "phase:far_field", "phase:jvp", "phase:vjp"};
std::mutex g_mu;
std::vector<Rec> g_recs;
std::vector<hipEvent_t> g_pool;
size_t g_used = 0;

const char* const KIND_NAMES[KIND_COUNT] = {"zgemm", "cgemm", "gj_panel",       "tp_select",
                                             "tp_exchange", "gj_permute",     "gather_scatter",
                                             "leaf_assemble", "pointwise"};

hipEvent_t take() {
  if (g_used == g_pool.size()) {
    hipEvent_t e;
    if (hipEventCreate(&e) != hipSuccess) return nullptr;
    g_pool.push_back(e);
  }
  return g_pool[g_used++];
}

}  // namespace

KernelTimer::KernelTimer(hipStream_t st, int kind, double flops, double bytes) {
  st_ = st;
  idx_ = -1;
  if (!g_on.load(std::memory_order_relaxed) || no_alloc_active()) return;
  std::lock_guard<std::mutex> lk(g_mu);
  hipEvent_t a = take(), b = take();
  if (!a || !b) return;
  if (hipEventRecord(a, st) != hipSuccess) return;
  g_recs.push_back(Rec{a, b, kind, g_phase.load(std::memory_order_relaxed), flops, bytes});
  idx_ = (long)g_recs.size() - 1;
}

KernelTimer::~KernelTimer() {
  if (idx_ < 0) return;
  std::lock_guard<std::mutex> lk(g_mu);
  if (idx_ < (long)g_recs.size()) (void)hipEventRecord(g_recs[idx_].b, st_);
}

void profile_set_phase(int phase) { g_phase.store(phase, std::memory_order_relaxed); }

bool profile_active() { return g_on.load(); }

}  // namespace hps

extern "C" {

hps_status hps_profile_start(void) {
  std::lock_guard<std::mutex> lk(hps::g_mu);
  hps::g_recs.clear();
  hps::g_used = 0;
  hps::g_on.store(true);
  return HPS_OK;
}

int hps_profile_stop(hps_kernel_stat* out, int max) {
  hps::g_on.store(false);
  if (hipDeviceSynchronize() != hipSuccess) return HPS_EDEVICE;
  std::lock_guard<std::mutex> lk(hps::g_mu);
  hps_kernel_stat acc[hps::KIND_COUNT], ph[hps::PHASE_COUNT];
  std::memset(acc, 0, sizeof(acc));
  std::memset(ph, 0, sizeof(ph));
  for (int k = 0; k < hps::KIND_COUNT; ++k)
    std::strncpy(acc[k].name, hps::KIND_NAMES[k], sizeof(acc[k].name) - 1);
  for (int k = 0; k < hps::PHASE_COUNT; ++k)
    std::strncpy(ph[k].name, hps::PHASE_NAMES[k], sizeof(ph[k].name) - 1);
  for (const auto& r : hps::g_recs) {
    float ms = 0.0f;
    if (hipEventElapsedTime(&ms, r.a, r.b) != hipSuccess) continue;
    for (hps_kernel_stat* s : {&acc[r.kind], &ph[r.phase]}) {
      s->launches += 1;
      s->total_ms += ms;
      s->flops += r.flops;
      s->bytes += r.bytes;
    }
  }
  int n = 0;
  for (int k = 0; k < hps::KIND_COUNT && n < max; ++k)
    if (acc[k].launches > 0 && out) out[n++] = acc[k];
  for (int k = 0; k < hps::PHASE_COUNT && n < max; ++k)
    if (ph[k].launches > 0 && out) out[n++] = ph[k];
  hps::g_recs.clear();
  hps::g_used = 0;
  return n;
}

}  // extern "C"
