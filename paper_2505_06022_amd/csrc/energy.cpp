// Device energy, read the way the paper's SYnergy queue exposes it (section
// 4, third listing: whole-device energy, and a kernel's energy as the
// difference around it), through the vendor interface for AMD GPUs.
//
// Backends, chosen on first use (or forced with CCL_ENERGY_BACKEND):
//   counter : amd-smi's cumulative energy accumulator (resolution in uJ)
//   power   : amd-smi's current socket power, integrated by a sampling
//             thread every 5 ms (for machines where the accumulator is not
//             exposed, e.g. virtual machine guests)
//   fake    : a scripted counter for host-only tests: 250 W times the time
//             since the first read (never chosen automatically)
// libamd_smi is opened at run time so the library loads without it.
#include <amd_smi/amdsmi.h>
#include <dlfcn.h>

#include <atomic>
#include <chrono>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <mutex>
#include <string>
#include <thread>
#include <vector>

#include "ccl_internal.h"

namespace ccl {
namespace {

using fn_init = amdsmi_status_t (*)(uint64_t);
using fn_sockets = amdsmi_status_t (*)(uint32_t *, amdsmi_socket_handle *);
using fn_procs = amdsmi_status_t (*)(amdsmi_socket_handle, uint32_t *, amdsmi_processor_handle *);
using fn_bdf = amdsmi_status_t (*)(amdsmi_processor_handle, amdsmi_bdf_t *);
using fn_energy = amdsmi_status_t (*)(amdsmi_processor_handle, uint64_t *, float *, uint64_t *);
using fn_power = amdsmi_status_t (*)(amdsmi_processor_handle, amdsmi_power_info_t *);

enum Backend { kNone = 0, kCounter = 1, kPower = 2, kFake = 3 };

struct Sampler {
  std::thread th;
  std::atomic<bool> stop{false};
  std::atomic<double> joules{0.0};
  std::atomic<uint64_t> stamp_ns{0};
};

struct DeviceEnergy {
  bool probed = false;
  Backend backend = kNone;
  amdsmi_processor_handle handle = nullptr;
  Sampler *sampler = nullptr;
  std::string why;
};

struct Smi {
  std::mutex mu;
  bool loaded = false;
  bool ok = false;
  std::string why;
  void *dl = nullptr;
  fn_init init = nullptr;
  fn_sockets sockets = nullptr;
  fn_procs procs = nullptr;
  fn_bdf bdf = nullptr;
  fn_energy energy = nullptr;
  fn_power power = nullptr;
  std::vector<amdsmi_processor_handle> gpus;
  std::vector<DeviceEnergy> dev;
  std::chrono::steady_clock::time_point fake_t0;
  bool fake_started = false;
};

Smi &smi() {
  static Smi *s = new Smi();  // never destroyed: sampler threads may outlive statics
  return *s;
}

uint64_t now_ns() {
  return static_cast<uint64_t>(std::chrono::duration_cast<std::chrono::nanoseconds>(
                                   std::chrono::steady_clock::now().time_since_epoch())
                                   .count());
}

bool load_smi(Smi &s) {
  if (s.loaded) return s.ok;
  s.loaded = true;
  s.dl = dlopen("libamd_smi.so", RTLD_NOW | RTLD_LOCAL);
  if (!s.dl) s.dl = dlopen("/opt/rocm/lib/libamd_smi.so", RTLD_NOW | RTLD_LOCAL);
  if (!s.dl) {
    s.why = "libamd_smi.so not found";
    return false;
  }
  s.init = reinterpret_cast<fn_init>(dlsym(s.dl, "amdsmi_init"));
  s.sockets = reinterpret_cast<fn_sockets>(dlsym(s.dl, "amdsmi_get_socket_handles"));
  s.procs = reinterpret_cast<fn_procs>(dlsym(s.dl, "amdsmi_get_processor_handles"));
  s.bdf = reinterpret_cast<fn_bdf>(dlsym(s.dl, "amdsmi_get_gpu_device_bdf"));
  s.energy = reinterpret_cast<fn_energy>(dlsym(s.dl, "amdsmi_get_energy_count"));
  s.power = reinterpret_cast<fn_power>(dlsym(s.dl, "amdsmi_get_power_info"));
  if (!s.init || !s.sockets || !s.procs) {
    s.why = "amd-smi symbols missing";
    return false;
  }
  if (s.init(AMDSMI_INIT_AMD_GPUS) != AMDSMI_STATUS_SUCCESS) {
    s.why = "amdsmi_init failed";
    return false;
  }
  uint32_t ns = 0;
  if (s.sockets(&ns, nullptr) != AMDSMI_STATUS_SUCCESS || ns == 0) {
    s.why = "no amd-smi sockets";
    return false;
  }
  std::vector<amdsmi_socket_handle> socks(ns);
  if (s.sockets(&ns, socks.data()) != AMDSMI_STATUS_SUCCESS) {
    s.why = "amdsmi_get_socket_handles failed";
    return false;
  }
  for (uint32_t i = 0; i < ns; ++i) {
    uint32_t np = 0;
    if (s.procs(socks[i], &np, nullptr) != AMDSMI_STATUS_SUCCESS || np == 0) continue;
    std::vector<amdsmi_processor_handle> ps(np);
    if (s.procs(socks[i], &np, ps.data()) != AMDSMI_STATUS_SUCCESS) continue;
    for (uint32_t j = 0; j < np; ++j) s.gpus.push_back(ps[j]);
  }
  if (s.gpus.empty()) {
    s.why = "amd-smi sees no GPU";
    return false;
  }
  s.ok = true;
  return true;
}

// amd-smi handle of HIP device `device`, matched by PCI address.
amdsmi_processor_handle match_handle(Smi &s, int device) {
  char bus[64] = {0};
  if (hipDeviceGetPCIBusId(bus, sizeof(bus), device) == hipSuccess && s.bdf) {
    unsigned dom = 0, b = 0, d = 0, f = 0;
    if (sscanf(bus, "%x:%x:%x.%x", &dom, &b, &d, &f) == 4) {
      for (auto h : s.gpus) {
        amdsmi_bdf_t x;
        memset(&x, 0, sizeof(x));
        if (s.bdf(h, &x) != AMDSMI_STATUS_SUCCESS) continue;
        if (x.domain_number == dom && x.bus_number == b && x.device_number == d &&
            x.function_number == f)
          return h;
      }
    }
  }
  if (s.gpus.size() == 1) return s.gpus[0];
  return nullptr;
}

double power_watts(Smi &s, amdsmi_processor_handle h, bool *ok) {
  amdsmi_power_info_t pi;
  memset(&pi, 0, sizeof(pi));
  *ok = false;
  if (!s.power || s.power(h, &pi) != AMDSMI_STATUS_SUCCESS) return 0.0;
  if (pi.current_socket_power != 0 && pi.current_socket_power != UINT32_MAX) {
    *ok = true;
    return static_cast<double>(pi.current_socket_power);
  }
  if (pi.average_socket_power != 0 && pi.average_socket_power != UINT32_MAX) {
    *ok = true;
    return static_cast<double>(pi.average_socket_power);
  }
  if (pi.socket_power != 0 && pi.socket_power != UINT32_MAX && pi.socket_power != UINT64_MAX) {
    *ok = true;
    return static_cast<double>(pi.socket_power);
  }
  return 0.0;
}

void sampler_loop(Sampler *sp, amdsmi_processor_handle h) {
  Smi &s = smi();
  uint64_t last = now_ns();
  bool ok = false;
  double w_last = power_watts(s, h, &ok);
  while (!sp->stop.load()) {
    std::this_thread::sleep_for(std::chrono::milliseconds(5));
    const uint64_t t = now_ns();
    const double w = power_watts(s, h, &ok);
    // trapezoid rule between samples
    const double dt = static_cast<double>(t - last) * 1e-9;
    double j = sp->joules.load();
    sp->joules.store(j + 0.5 * (w + w_last) * dt);
    sp->stamp_ns.store(t);
    last = t;
    w_last = w;
  }
}

ccl_status probe(Smi &s, int device, DeviceEnergy &de) {
  de.probed = true;
  const char *force = getenv("CCL_ENERGY_BACKEND");
  const std::string want = force ? force : "";
  if (want == "fake") {
    de.backend = kFake;
    return CCL_OK;
  }
  if (!load_smi(s)) {
    de.why = s.why;
    return CCL_E_UNSUPPORTED;
  }
  de.handle = match_handle(s, device);
  if (!de.handle) {
    de.why = "no amd-smi GPU matches the HIP device's PCI address";
    return CCL_E_UNSUPPORTED;
  }
  if (want.empty() || want == "counter") {
    uint64_t acc = 0, ts = 0;
    float res = 0.0f;
    if (s.energy && s.energy(de.handle, &acc, &res, &ts) == AMDSMI_STATUS_SUCCESS && res > 0.0f) {
      de.backend = kCounter;
      return CCL_OK;
    }
    if (want == "counter") {
      de.why = "amdsmi_get_energy_count not supported here";
      return CCL_E_UNSUPPORTED;
    }
  }
  bool ok = false;
  power_watts(s, de.handle, &ok);
  if (!ok) {
    de.why = "neither the energy counter nor socket power is available";
    return CCL_E_UNSUPPORTED;
  }
  de.backend = kPower;
  de.sampler = new Sampler();
  de.sampler->stamp_ns.store(now_ns());
  de.sampler->th = std::thread(sampler_loop, de.sampler, de.handle);
  de.sampler->th.detach();
  return CCL_OK;
}

}  // namespace
}  // namespace ccl

using namespace ccl;

extern "C" ccl_status ccl_energy_read(int32_t device, void *hip_stream, double *joules,
                                      uint64_t *timestamp_ns) {
  clear_error();
  if (!joules) return fail(CCL_E_INVALID, "joules is NULL");
  if (device < 0) return fail(CCL_E_INVALID, "device < 0");
  if (hip_stream) {
    ccl_status st = hip_check(hipStreamSynchronize(static_cast<hipStream_t>(hip_stream)),
                              "hipStreamSynchronize");
    if (st != CCL_OK) return st;
  }
  Smi &s = smi();
  std::lock_guard<std::mutex> lock(s.mu);
  if (s.dev.size() <= static_cast<size_t>(device)) s.dev.resize(device + 1);
  DeviceEnergy &de = s.dev[device];
  if (!de.probed) {
    ccl_status st = probe(s, device, de);
    if (st != CCL_OK) return fail(st, "energy: %s", de.why.c_str());
  }
  switch (de.backend) {
    case kCounter: {
      uint64_t acc = 0, ts = 0;
      float res = 0.0f;
      if (s.energy(de.handle, &acc, &res, &ts) != AMDSMI_STATUS_SUCCESS)
        return fail(CCL_E_UNSUPPORTED, "amdsmi_get_energy_count failed");
      *joules = static_cast<double>(acc) * static_cast<double>(res) * 1e-6;
      if (timestamp_ns) *timestamp_ns = ts;
      return CCL_OK;
    }
    case kPower:
      *joules = de.sampler->joules.load();
      if (timestamp_ns) *timestamp_ns = de.sampler->stamp_ns.load();
      return CCL_OK;
    case kFake: {
      if (!s.fake_started) {
        s.fake_started = true;
        s.fake_t0 = std::chrono::steady_clock::now();
      }
      const double t = std::chrono::duration<double>(std::chrono::steady_clock::now() - s.fake_t0)
                           .count();
      *joules = 250.0 * t;
      if (timestamp_ns) *timestamp_ns = now_ns();
      return CCL_OK;
    }
    default:
      return fail(CCL_E_UNSUPPORTED, "energy: %s", de.why.c_str());
  }
}

extern "C" const char *ccl_energy_backend(int32_t device) {
  Smi &s = smi();
  std::lock_guard<std::mutex> lock(s.mu);
  if (device < 0 || static_cast<size_t>(device) >= s.dev.size() || !s.dev[device].probed)
    return "unprobed";
  switch (s.dev[device].backend) {
    case kCounter: return "amdsmi-energy-counter";
    case kPower: return "amdsmi-power-integrated";
    case kFake: return "fake";
    default: return "unsupported";
  }
}
