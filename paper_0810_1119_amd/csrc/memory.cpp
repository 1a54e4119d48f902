// Device memory accounting: every allocation the library makes while a
// plan's entry point runs is recorded against that plan until it is freed,
// so that a caller can ask how much device memory a plan holds.
#include <mutex>
#include <unordered_map>

#include "engine.h"

namespace gabp {

namespace {

thread_local DevAccount *tl_account = nullptr;

struct Registry {
  std::mutex mu;
  std::unordered_map<void *, std::pair<size_t, DevAccount *>> live;
};

Registry &registry() {
  static Registry r;
  return r;
}

}  // namespace

AccountScope::AccountScope(DevAccount *a) : prev(tl_account) { tl_account = a; }
AccountScope::~AccountScope() { tl_account = prev; }

hipError_t dalloc_bytes(void **p, size_t bytes) {
  *p = nullptr;
  const hipError_t e = hipMalloc(p, bytes);
  if (e != hipSuccess || !tl_account) return e;
  Registry &r = registry();
  std::lock_guard<std::mutex> lock(r.mu);
  r.live[*p] = {bytes, tl_account};
  tl_account->bytes += (int64_t)bytes;
  return e;
}

void dfree(void *p) {
  if (!p) return;
  {
    Registry &r = registry();
    std::lock_guard<std::mutex> lock(r.mu);
    auto it = r.live.find(p);
    if (it != r.live.end()) {
      it->second.second->bytes -= (int64_t)it->second.first;
      r.live.erase(it);
    }
  }
  (void)hipFree(p);
}

}  // namespace gabp
