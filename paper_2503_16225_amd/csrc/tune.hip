// Autotuner of launch configurations.  Some kernels have several valid
// configurations with identical results, whose speed depends on the shape in
// use and on the chip: the tile shape of the complex block products (larger
// tiles read each operand fewer times, smaller ones fill the chip at small
// sizes), and the number of work-groups of the multi-work-group Householder
// reduction of large Hermitian matrices (fewer make each step's exchange
// cheaper, more bring more CUs' bandwidth).
//
// The table maps "<arch>/<CUs> <kernel> <shape class>" to the chosen
// candidate.  Mode 1 (tuning on): the first use of a class that the table
// lacks times every candidate on the stream (a warm-up launch and a timed
// one, on scratch outputs or copies, so the caller's data are untouched) and
// keeps the fastest for the rest of the process.  Mode 2: the table's
// choices are used and nothing is timed (classes it lacks take the default).
// Mode 0 (the default): candidate 0 everywhere.  Tables are saved and loaded
// as text; switching tuning on loads, once, the table file that sits beside
// the library (tune_table.txt), if there is one.
#include <dlfcn.h>

#include <atomic>
#include <fstream>
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
std::atomic<int> g_force{-1};
std::atomic<bool> g_default_loaded{false};
thread_local int g_hold = 0;

// "<arch>/<CUs>" of the current device (cached per device index)
std::string dev_tag() {
  static std::mutex mu;
  static std::map<int, std::string> tags;
  int dev = 0;
  HIPCK(hipGetDevice(&dev));
  std::lock_guard<std::mutex> lk(mu);
  auto it = tags.find(dev);
  if (it != tags.end()) return it->second;
  hipDeviceProp_t pr;
  HIPCK(hipGetDeviceProperties(&pr, dev));
  std::string arch = pr.gcnArchName;
  arch = arch.substr(0, arch.find(':'));
  const std::string t = arch + "/" + std::to_string(pr.multiProcessorCount);
  tags[dev] = t;
  return t;
}

std::string full_key(const std::string& key) { return dev_tag() + " " + key; }

std::string format_table() {
  std::ostringstream os;
  std::lock_guard<std::mutex> lk(g_mu);
  for (const auto& kv : g_table) {
    os << kv.first << ": choice " << kv.second.choice << " ms";
    for (float m : kv.second.ms) os << " " << m;
    os << "\n";
  }
  return os.str();
}

// Reads lines "<key>: choice <c> ms <t0> <t1> ..."; entries already in the
// table are kept.  Returns the number of entries added; -1 if the file
// cannot be opened; EAHP_EINVAL for a malformed line.
int load_table(const std::string& path) {
  std::ifstream f(path);
  if (!f) return -1;
  std::string line;
  int added = 0, lineno = 0;
  std::lock_guard<std::mutex> lk(g_mu);
  while (std::getline(f, line)) {
    ++lineno;
    if (line.empty() || line[0] == '#') continue;
    const size_t at = line.find(": choice ");
    if (at == std::string::npos)
      fail(EAHP_EINVAL, "autotune table " + path + ": line " + std::to_string(lineno) + " malformed");
    std::istringstream rest(line.substr(at + 9));
    Entry e;
    std::string word;
    if (!(rest >> e.choice) || e.choice < 0)
      fail(EAHP_EINVAL, "autotune table " + path + ": line " + std::to_string(lineno) + " has no valid choice");
    if (rest >> word && word == "ms") {
      float m;
      while (rest >> m) e.ms.push_back(m);
    }
    if (g_table.emplace(line.substr(0, at), e).second) ++added;
  }
  return added;
}

void load_default_once() {
  bool expect = false;
  if (!g_default_loaded.compare_exchange_strong(expect, true)) return;
  Dl_info info;
  if (!dladdr(reinterpret_cast<void*>(&load_default_once), &info) || !info.dli_fname) return;
  std::string p = info.dli_fname;
  const size_t slash = p.rfind('/');
  p = (slash == std::string::npos ? std::string(".") : p.substr(0, slash)) + "/tune_table.txt";
  (void)load_table(p);
}
}  // namespace

bool autotune_on() { return g_on.load() != 0; }
int autotune_forced() { return g_force.load(); }
AutotuneHold::AutotuneHold() { ++g_hold; }
AutotuneHold::~AutotuneHold() { --g_hold; }

int autotune_kept(const std::string& key) {
  if (!autotune_on()) return 0;
  const std::string k = full_key(key);
  std::lock_guard<std::mutex> lk(g_mu);
  auto it = g_table.find(k);
  return it != g_table.end() ? it->second.choice : 0;
}

int autotune(hipStream_t st, const std::string& key, int ncand, const std::function<void(int)>& run) {
  if (!autotune_on() || ncand <= 1) return 0;
  const std::string k = full_key(key);
  {
    std::lock_guard<std::mutex> lk(g_mu);
    auto it = g_table.find(k);
    if (it != g_table.end()) return std::min(it->second.choice, ncand - 1);
  }
  if (g_on.load() != 1 || g_hold > 0) return 0;
  hipStreamCaptureStatus cs = hipStreamCaptureStatusNone;
  HIPCK(hipStreamIsCapturing(st, &cs));
  if (cs != hipStreamCaptureStatusNone) return 0;
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

namespace {
template <typename F>
int tune_guarded(F&& f) {
  try {
    f();
    return EAHP_OK;
  } catch (const eahp::Error& e) {
    eahp::g_last_error = e.msg;
    return e.status;
  } catch (...) {
    eahp::g_last_error = "unknown error";
    return EAHP_EDEVICE;
  }
}
}  // namespace

extern "C" int eahp_autotune_enable(int mode) {
  if (mode < 0 || mode > 2) {
    eahp::g_last_error = "autotune mode must be 0, 1 or 2";
    return EAHP_EINVAL;
  }
  return tune_guarded([&] {
    if (mode != 0) eahp::load_default_once();
    eahp::g_on.store(mode);
  });
}

extern "C" int eahp_autotune_force(int choice) {
  eahp::g_force.store(choice < 0 ? -1 : choice);
  return EAHP_OK;
}

extern "C" int eahp_autotune_load(const char* path, int* added) {
  return tune_guarded([&] {
    if (!path) eahp::fail(EAHP_EINVAL, "null path");
    const int n = eahp::load_table(path);
    if (n < 0) eahp::fail(EAHP_EINVAL, std::string("cannot open autotune table ") + path);
    if (added) *added = n;
  });
}

extern "C" int eahp_autotune_save(const char* path) {
  return tune_guarded([&] {
    if (!path) eahp::fail(EAHP_EINVAL, "null path");
    std::ofstream f(path);
    if (!f) eahp::fail(EAHP_EINVAL, std::string("cannot write autotune table ") + path);
    f << eahp::format_table();
    if (!f) eahp::fail(EAHP_EINVAL, std::string("write failed: ") + path);
  });
}

extern "C" int eahp_autotune_report(char* buf, size_t len, size_t* needed) {
  const std::string s = eahp::format_table();
  if (needed) *needed = s.size() + 1;
  if (buf && len > 0) {
    const size_t n = std::min(len - 1, s.size());
    std::copy(s.begin(), s.begin() + n, buf);
    buf[n] = 0;
  }
  return EAHP_OK;
}
