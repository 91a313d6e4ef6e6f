// Serialises the graph capture of a lock-step batch against the library calls
// that allocate, free or synchronise device memory (a context's setup and
// destruction, the first block solve's allocation), whichever host threads make
// them. While a stream capture is open the HIP runtime records launches on the
// captured stream into a graph; a device-wide synchronisation or an allocation
// made meanwhile by another thread (hipFree synchronises the device) is outside
// what a capture supports. With this guard:
//   - a capture opens only when no such call is in progress; otherwise the
//     caller runs that step without a graph (try_begin_capture returns false);
//   - such a call waits while a capture is open (captures record a handful of
//     launches and end at once).
// Host-only code (no HIP): it is also compiled and exercised on the CPU.
#pragma once

#include <condition_variable>
#include <mutex>

namespace coarse {

class CaptureGuard {
 public:
  bool try_begin_capture() {
    std::lock_guard<std::mutex> lk(mu_);
    if (device_calls_ > 0) return false;
    ++captures_;
    return true;
  }
  void end_capture() {
    {
      std::lock_guard<std::mutex> lk(mu_);
      --captures_;
    }
    cv_.notify_all();
  }
  void begin_device_call() {
    std::unique_lock<std::mutex> lk(mu_);
    cv_.wait(lk, [&] { return captures_ == 0; });
    ++device_calls_;
  }
  void end_device_call() {
    std::lock_guard<std::mutex> lk(mu_);
    --device_calls_;
  }
  int captures() {
    std::lock_guard<std::mutex> lk(mu_);
    return captures_;
  }
  int device_calls() {
    std::lock_guard<std::mutex> lk(mu_);
    return device_calls_;
  }

 private:
  std::mutex mu_;
  std::condition_variable cv_;
  int captures_ = 0;
  int device_calls_ = 0;
};

// Holds a device call for the lifetime of the object.
class DeviceCallScope {
 public:
  explicit DeviceCallScope(CaptureGuard &g) : g_(g) { g_.begin_device_call(); }
  ~DeviceCallScope() { g_.end_device_call(); }
  DeviceCallScope(const DeviceCallScope &) = delete;
  DeviceCallScope &operator=(const DeviceCallScope &) = delete;

 private:
  CaptureGuard &g_;
};

}  // namespace coarse
