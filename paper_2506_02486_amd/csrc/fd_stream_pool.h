// fd_stream_pool.h -- a bounded pool of streams (host-only policy; the stream
// operations are a template parameter, so the policy is tested on the host with
// simulated streams).
//
// The paper's runtime manages the streams of its asynchronous work (Sec. 3.2):
// streams are created on demand, idle ones are reused, and at most
// MAX_ACTIVE_STREAMS are active; when the bound is reached only half of the
// streams whose work has completed are synchronised and released, while the other
// active streams keep running.  The shot server runs each shot's admission work
// (zeroing, the max(v) reduction, model preparation, table uploads) on a stream
// from such a pool, so that admissions overlap one another and the steps queued on
// the compute stream.
//
// Ops must provide: typename Stream; bool create(Stream*) (false: could not);
// bool done(Stream) (all work enqueued on it so far has completed); void
// sync(Stream) (wait for that work); void destroy(Stream).
#pragma once

#include <deque>
#include <vector>

namespace fd {

template <class Ops>
class StreamPool {
 public:
  using Stream = typename Ops::Stream;

  StreamPool(Ops ops, int max_active) : ops_(ops), max_(max_active < 1 ? 1 : max_active) {}
  StreamPool(const StreamPool&) = delete;
  StreamPool& operator=(const StreamPool&) = delete;
  ~StreamPool() { shutdown(); }

  // A stream for new work, counted active until a partial synchronisation releases
  // it: an idle stream if there is one (reuse); else a new one while fewer than the
  // bound exist (lazy creation); else partial synchronisation -- of the active
  // streams whose work has completed, the older half (rounded up) is released to
  // the idle list and the oldest of them handed out (done() has already shown their
  // work complete: they need no wait); if none has completed, the oldest active
  // stream is synchronised (this call then waits for its work) and handed out.
  // *created and *synced (may be NULL) report what the call did: *synced is the
  // number of streams released.  Returns false only if a stream could not be
  // created.
  bool acquire(Stream* out, bool* created = nullptr, int* synced = nullptr) {
    if (created) *created = false;
    if (synced) *synced = 0;
    if (idle_.empty()) {
      if ((int)active_.size() < max_) {
        Stream s;
        if (!ops_.create(&s)) return false;
        if (created) *created = true;
        idle_.push_back(s);
      } else {
        const int n = partial_sync();
        if (synced) *synced = n;
      }
    }
    *out = idle_.front();
    idle_.pop_front();
    active_.push_back(*out);
    return true;
  }

  // Synchronise and release every active stream (their work finished); the streams
  // stay in the pool for reuse.
  void sync_all() {
    for (const Stream& s : active_) {
      ops_.sync(s);
      idle_.push_back(s);
    }
    active_.clear();
  }

  // Synchronise and destroy every stream.
  void shutdown() {
    sync_all();
    for (const Stream& s : idle_) ops_.destroy(s);
    idle_.clear();
  }

  int active() const { return (int)active_.size(); }
  int idle() const { return (int)idle_.size(); }
  int live() const { return (int)(active_.size() + idle_.size()); }
  int bound() const { return max_; }
  // Active streams, oldest first.
  const std::deque<Stream>& active_streams() const { return active_; }

 private:
  // Release the older half (rounded up) of the completed active streams; if none
  // has completed, wait for the oldest (the only case that calls sync).  Returns
  // the number released.
  int partial_sync() {
    std::vector<size_t> done;
    for (size_t i = 0; i < active_.size(); ++i)
      if (ops_.done(active_[i])) done.push_back(i);
    std::vector<size_t> take;
    if (done.empty()) {
      take.push_back(0);
      ops_.sync(active_[0]);
    } else {
      const size_t half = (done.size() + 1) / 2;
      take.assign(done.begin(), done.begin() + half);
    }
    std::deque<Stream> keep;
    size_t t = 0;
    for (size_t i = 0; i < active_.size(); ++i) {
      if (t < take.size() && take[t] == i) {
        idle_.push_back(active_[i]);
        ++t;
      } else {
        keep.push_back(active_[i]);
      }
    }
    active_.swap(keep);
    return (int)take.size();
  }

  Ops ops_;
  int max_;
  std::deque<Stream> active_;  // in order of acquisition
  std::deque<Stream> idle_;
};

}  // namespace fd
