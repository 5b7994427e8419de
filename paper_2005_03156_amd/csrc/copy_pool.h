// A few host threads that share out memory copies (used by the served form
// to pack request pieces into its pinned pool and results out of it).
// Plain C++: no device code, so it is also built and tested on its own.
#pragma once

#include <algorithm>
#include <atomic>
#include <condition_variable>
#include <cstring>
#include <deque>
#include <mutex>
#include <thread>
#include <vector>

namespace bm {

// run() hands its copies to the workers, takes part itself, and returns when
// all are done; several threads may call it at the same time. A pool of one
// thread copies on the caller's thread alone.
class CopyPool {
 public:
  struct Copy {
    const void* src;
    void* dst;
    size_t bytes;
  };
  explicit CopyPool(int threads) {
    for (int i = 1; i < threads; ++i) th_.emplace_back([this] { work(); });
  }
  ~CopyPool() {
    {
      std::lock_guard<std::mutex> g(mu_);
      stop_ = true;
    }
    cv_.notify_all();
    for (auto& t : th_) t.join();
  }
  // Copies of more than kSplit bytes are cut so that the threads share them.
  void run(const std::vector<Copy>& copies) {
    if (copies.empty()) return;
    Batch b;
    for (const Copy& c : copies)
      for (size_t o = 0; o < c.bytes; o += kSplit)
        b.items.push_back(Copy{static_cast<const char*>(c.src) + o, static_cast<char*>(c.dst) + o,
                               std::min(kSplit, c.bytes - o)});
    b.left = b.items.size();
    if (th_.empty() || b.items.size() == 1) {
      for (const Copy& c : b.items) memcpy(c.dst, c.src, c.bytes);
      return;
    }
    {
      std::lock_guard<std::mutex> g(mu_);
      q_.push_back(&b);
    }
    cv_.notify_all();
    drain(b);
    // b lives on this stack: wait until no worker holds it any more
    std::unique_lock<std::mutex> lk(mu_);
    done_.wait(lk, [&] { return b.left == 0 && b.users == 0; });
  }

 private:
  static constexpr size_t kSplit = (size_t)1 << 20;
  struct Batch {
    std::vector<Copy> items;
    std::atomic<size_t> next{0};
    size_t left = 0;  // items not yet copied (guarded by mu_)
    int users = 0;    // workers inside drain() for this batch (guarded by mu_)
  };
  // Take items of b until none is left; the last finisher wakes run().
  void drain(Batch& b) {
    size_t did = 0;
    for (size_t i; (i = b.next.fetch_add(1)) < b.items.size();) {
      memcpy(b.items[i].dst, b.items[i].src, b.items[i].bytes);
      ++did;
    }
    if (!did) return;
    std::lock_guard<std::mutex> g(mu_);
    b.left -= did;
    if (b.left == 0) {
      q_.erase(std::remove(q_.begin(), q_.end(), &b), q_.end());
      done_.notify_all();
    }
  }
  void work() {
    std::unique_lock<std::mutex> lk(mu_);
    for (;;) {
      cv_.wait(lk, [&] {
        if (stop_) return true;
        for (Batch* b : q_)
          if (b->next.load() < b->items.size()) return true;
        return false;
      });
      if (stop_) return;
      Batch* b = nullptr;
      for (Batch* x : q_)
        if (x->next.load() < x->items.size()) { b = x; break; }
      if (!b) continue;  // taken meanwhile by threads in drain(), which advance `next` without the lock
      ++b->users;
      lk.unlock();
      drain(*b);
      lk.lock();
      if (--b->users == 0 && b->left == 0) done_.notify_all();
    }
  }
  std::mutex mu_;
  std::condition_variable cv_, done_;
  std::deque<Batch*> q_;
  std::vector<std::thread> th_;
  bool stop_ = false;
};

}  // namespace bm
