// Autotuner of launch configurations.  Some kernels have several valid
// configurations whose speed depends on the shape in use and on the chip: the
// number of work-groups of the cooperative Householder reduction of the
// projected FOM systems (columns per work-group: fewer work-groups make the
// per-step grid barrier cheaper, more of them bring more CUs' bandwidth), and
// the split of the row dimension of the Gram products (more splits fill the
// chip, fewer write fewer partial tiles).  When tuning is on, the first use
// of a shape bucket times every candidate on the stream (a warm-up launch and
// a timed one, on scratch copies, so the caller's data are untouched) and
// keeps the fastest for the rest of the process; later uses take the kept
// choice.  When it is off, the default configuration (candidate 0) is used.
#include <atomic>
#include <map>
#include <mutex>
#include <sstream>

#include "ops.h"

namespace eahp {

namespace {
struct Entry {
  int choice = 0;
  std::vector<float> ms;
};
std::mutex g_mu;
std::map<std::string, Entry> g_table;
std::atomic<int> g_on{0};
}  // namespace

bool autotune_on() { return g_on.load() != 0; }

int autotune(hipStream_t st, const std::string& key, int ncand, const std::function<void(int)>& run) {
  if (!autotune_on() || ncand <= 1) return 0;
  int dev = 0;
  HIPCK(hipGetDevice(&dev));
  const std::string k = "dev" + std::to_string(dev) + " " + key;
  {
    std::lock_guard<std::mutex> lk(g_mu);
    auto it = g_table.find(k);
    if (it != g_table.end()) return it->second.choice;
  }
  hipEvent_t a, b;
  HIPCK(hipEventCreate(&a));
  HIPCK(hipEventCreate(&b));
  Entry e;
  float best = 0;
  for (int c = 0; c < ncand; ++c) {
    run(c);  // warm-up
    HIPCK(hipEventRecord(a, st));
    run(c);
    HIPCK(hipEventRecord(b, st));
    HIPCK(hipEventSynchronize(b));
    float ms = 0;
    HIPCK(hipEventElapsedTime(&ms, a, b));
    e.ms.push_back(ms);
    if (c == 0 || ms < best) {
      best = ms;
      e.choice = c;
    }
  }
  HIPCK(hipEventDestroy(a));
  HIPCK(hipEventDestroy(b));
  std::lock_guard<std::mutex> lk(g_mu);
  g_table[k] = e;
  return e.choice;
}

}  // namespace eahp

extern "C" int eahp_autotune_enable(int on) {
  eahp::g_on.store(on ? 1 : 0);
  return EAHP_OK;
}

extern "C" int eahp_autotune_report(char* buf, size_t len, size_t* needed) {
  std::ostringstream os;
  {
    std::lock_guard<std::mutex> lk(eahp::g_mu);
    for (const auto& kv : eahp::g_table) {
      os << kv.first << ": choice " << kv.second.choice << " ms";
      for (float m : kv.second.ms) os << " " << m;
      os << "\n";
    }
  }
  const std::string s = os.str();
  if (needed) *needed = s.size() + 1;
  if (buf && len > 0) {
    const size_t n = std::min(len - 1, s.size());
    std::copy(s.begin(), s.begin() + n, buf);
    buf[n] = 0;
  }
  return EAHP_OK;
}
