// Library-wide C ABI pieces: error strings, version, kernel-timing events.
#include <atomic>
#include <cstdarg>
#include <cstdlib>
#include <cstring>
#include <mutex>
#include <vector>

#include "common.hpp"

namespace sh {

static thread_local char g_err[512] = "";

void set_error(const char* fmt, ...) {
  va_list ap;
  va_start(ap, fmt);
  vsnprintf(g_err, sizeof(g_err), fmt, ap);
  va_end(ap);
}

const char* last_error() { return g_err; }

Arena*& arena_slot() {
  static thread_local Arena* a = nullptr;
  return a;
}

hipStream_t& upload_stream() {
  static thread_local hipStream_t s = nullptr;
  return s;
}

namespace {
std::atomic<int64_t> g_dev_live{0};

int64_t dev_cap() {   // SH_MAX_DEVICE_BYTES, read at every allocation so that it can change at run time
  const char* e = std::getenv("SH_MAX_DEVICE_BYTES");
  if (!e || !*e) return -1;
  char* end = nullptr;
  const long long v = std::strtoll(e, &end, 10);
  return (end && *end == '\0' && v > 0) ? int64_t(v) : -1;
}
}  // namespace

bool dev_reserve(size_t bytes) {
  const int64_t cap = dev_cap();
  const int64_t after = g_dev_live.fetch_add(int64_t(bytes)) + int64_t(bytes);
  if (cap > 0 && after > cap) {
    g_dev_live.fetch_sub(int64_t(bytes));
    return false;
  }
  return true;
}

void dev_unreserve(size_t bytes) { g_dev_live.fetch_sub(int64_t(bytes)); }

namespace {
const char* kNames[] = {"degrid", "grid", "fold", "fft_rows", "fft_cols", "dwt", "prox", "cg", "toeplitz"};
constexpr int kSlots = sizeof(kNames) / sizeof(kNames[0]);
struct Pending {
  hipEvent_t a, b;
  int slot;
};
std::mutex g_mu;
bool g_on = false;
std::vector<Pending> g_pending;
int64_t g_count[kSlots];
double g_ms[kSlots];

int slot_of(const char* name) {
  for (int i = 0; i < kSlots; ++i)
    if (std::strcmp(kNames[i], name) == 0) return i;
  return -1;
}

void drain_locked() {
  for (auto& p : g_pending) {
    float ms = 0.f;
    if (hipEventSynchronize(p.b) == hipSuccess && hipEventElapsedTime(&ms, p.a, p.b) == hipSuccess) {
      g_count[p.slot] += 1;
      g_ms[p.slot] += ms;
    }
    (void)hipEventDestroy(p.a);
    (void)hipEventDestroy(p.b);
  }
  g_pending.clear();
}
}  // namespace

bool profiling_on() { return g_on; }

ProfScope::ProfScope(const char* name, hipStream_t stream) : st(stream) {
  if (!g_on) return;
  slot = slot_of(name);
  if (slot < 0) return;
  if (hipEventCreate(&a) != hipSuccess || hipEventCreate(&b) != hipSuccess) {
    slot = -1;
    return;
  }
  (void)hipEventRecord(a, st);
}

ProfScope::~ProfScope() {
  if (slot < 0) return;
  (void)hipEventRecord(b, st);
  std::lock_guard<std::mutex> g(g_mu);
  g_pending.push_back({a, b, slot});
  if (g_pending.size() > 4096) drain_locked();
}

}  // namespace sh

extern "C" {

const char* sh_last_error(void) { return sh::last_error(); }

const char* sh_version(void) { return "sarahip 0.1 (gfx950)"; }

sh_status sh_device_bytes(int64_t* live_bytes, int64_t* cap_bytes) {
  SH_REQUIRE(live_bytes || cap_bytes, "NULL argument");
  if (live_bytes) *live_bytes = sh::g_dev_live.load();
  if (cap_bytes) *cap_bytes = sh::dev_cap();
  return SH_OK;
}

sh_status sh_profile_enable(int32_t on) {
  std::lock_guard<std::mutex> g(sh::g_mu);
  sh::drain_locked();
  for (int i = 0; i < sh::kSlots; ++i) {
    sh::g_count[i] = 0;
    sh::g_ms[i] = 0.0;
  }
  sh::g_on = on != 0;
  return SH_OK;
}

sh_status sh_profile_read(const char* name, int64_t* count, double* total_ms) {
  SH_REQUIRE(name && count && total_ms, "NULL argument");
  std::lock_guard<std::mutex> g(sh::g_mu);
  const int s = sh::slot_of(name);
  SH_REQUIRE(s >= 0, "unknown kernel name '%s'", name);
  sh::drain_locked();
  *count = sh::g_count[s];
  *total_ms = sh::g_ms[s];
  return SH_OK;
}

}  // extern "C"
