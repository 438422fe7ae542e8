// Sanitizer driver for the host side of the C ABI (test infrastructure):
// fs_api.cpp compiled for the host only, under AddressSanitizer and
// UndefinedBehaviorSanitizer, driven through every validation path that runs
// before a device is touched (sizes, options, NULL arguments), the workspace
// size computation for every supported configuration, and plan creation on a
// machine without a device.  The solvers' ops tables live in the kernel
// translation units; here they are stand-ins with the same shape of answer
// (an ops table with element counts for supported sizes, none otherwise).
// Any out-of-bounds access or undefined operation aborts the run.
#include <cmath>
#include <cstdio>
#include <cstdlib>

#include "fs.h"
#include "fs_internal.h"

namespace fs {
namespace {
void stand_in_stage(Plan*, void*, int, int) {}
Ops stand_in(int n, int nfield, int ndim) {
  Ops o{};
  if (n < 16 || n > 1024 || (n & (n - 1))) return o;
  const size_t plane = (size_t)n * (n / 2 + 1) * (ndim == 3 ? (size_t)n : 1);
  o.stage = stand_in_stage;
  o.elems_a = 7 * plane;
  o.elems_b = 7 * plane;
  o.elems_acc = (size_t)nfield * plane;
  o.elems_full = plane;
  o.elems_sin = ndim == 2 && nfield == 2 ? 2 * plane : 0;
  return o;
}
}  // namespace
template <typename T>
Ops make_ops3(int n, int nfield) {
  return stand_in(n, nfield, 3);
}
template <typename T>
Ops make_ops2(int n, int nfield) {
  return stand_in(n, nfield, 2);
}
template Ops make_ops3<float>(int, int);
template Ops make_ops3<double>(int, int);
template Ops make_ops2<float>(int, int);
template Ops make_ops2<double>(int, int);
void launch_time(Plan*, double*, double*) {}
}  // namespace fs

static int failures = 0;

static void expect(fs_status got, fs_status want, const char* what) {
  if (got != want) {
    std::printf("FAIL %s: status %d (%s), expected %d: %s\n", what, (int)got, fs_status_str(got),
                (int)want, fs_last_error());
    failures++;
  }
}

int main() {
  for (int s = 1; s >= -6; s--) (void)fs_status_str((fs_status)s);
  (void)fs_last_error();

  // workspace sizes of every supported configuration, without a device
  for (int ndim = 2; ndim <= 3; ndim++)
    for (int prec = FS_F32; prec <= FS_F64; prec++)
      for (int bous = 0; bous <= 1; bous++)
        for (int n = 16; n <= 1024; n *= 2) {
          fs_plan_opts o;
          fs_plan_opts_default(&o);
          o.ndim = ndim;
          o.precision = prec;
          o.flags = bous ? FS_BOUSSINESQ : 0u;
          if (ndim == 3 && !bous) o.forcing_power = 5e-3;
          size_t bytes = 0;
          const fs_status st = fs_plan_workspace_bytes(n, &o, &bytes);
          const bool ok = !(ndim == 3 && prec == FS_F64 && n > 512);
          expect(st, ok ? FS_OK : FS_E_UNSUPPORTED, "workspace bytes");
          if (ok && bytes == 0) {
            std::printf("FAIL zero workspace\n");
            failures++;
          }
        }
  size_t bytes;
  expect(fs_plan_workspace_bytes(64, nullptr, nullptr), FS_E_INVALID, "NULL bytes");
  expect(fs_plan_workspace_bytes(48, nullptr, &bytes), FS_E_UNSUPPORTED, "n = 48");

  // plan creation: invalid arguments are rejected before any device call
  fs_plan* plan = nullptr;
  fs_plan_opts o;
  fs_plan_opts_default(&o);
  expect(fs_plan_create(nullptr, 64, 6.28, 0.1, 0.01, &o), FS_E_INVALID, "NULL out");
  expect(fs_plan_create(&plan, 0, 6.28, 0.1, 0.01, &o), FS_E_INVALID, "n = 0");
  expect(fs_plan_create(&plan, 2048, 6.28, 0.1, 0.01, &o), FS_E_UNSUPPORTED, "n = 2048");
  expect(fs_plan_create(&plan, 64, NAN, 0.1, 0.01, &o), FS_E_INVALID, "L = nan");
  expect(fs_plan_create(&plan, 64, 6.28, -1.0, 0.01, &o), FS_E_INVALID, "nu < 0");
  expect(fs_plan_create(&plan, 64, 6.28, 0.1, INFINITY, &o), FS_E_INVALID, "dt = inf");
  fs_plan_opts b = o;
  b.flags = 0x100u;
  expect(fs_plan_create(&plan, 64, 6.28, 0.1, 0.01, &b), FS_E_INVALID, "flags");
  b = o;
  b.forcing_power = 1.0;
  b.forcing_kmax = 1e300;
  expect(fs_plan_create(&plan, 64, 6.28, 0.1, 0.01, &b), FS_E_INVALID, "band");
  b = o;
  b.workspace = (void*)0x1001;
  b.workspace_bytes = 1 << 20;
  expect(fs_plan_create(&plan, 64, 6.28, 0.1, 0.01, &b), FS_E_INVALID, "workspace");
  // a valid plan on a machine without a device: FS_E_DEVICE, nothing created
  const fs_status st = fs_plan_create(&plan, 32, 6.28, 0.1, 0.01, &o);
  if (st == FS_OK) {
    fs_plan_destroy(plan);  // a device exists after all
  } else {
    expect(st, FS_E_DEVICE, "no device");
    if (plan) {
      std::printf("FAIL plan set on error\n");
      failures++;
    }
  }
  // calls on a NULL plan
  expect(fs_plan_destroy(nullptr), FS_OK, "destroy NULL");
  expect(fs_step_rk4(nullptr, nullptr, 1), FS_E_INVALID, "step NULL plan");
  expect(fs_tendency(nullptr, nullptr, nullptr), FS_E_INVALID, "tendency NULL plan");
  expect(fs_energy_spectrum(nullptr, nullptr, nullptr, 8, nullptr, nullptr), FS_E_INVALID,
         "spectrum NULL plan");
  size_t elems;
  expect(fs_state_elems(nullptr, &elems), FS_E_INVALID, "elems NULL plan");

  std::printf("abi sanitizer run: %s (%d failures)\n", failures ? "FAILED" : "ok", failures);
  return failures ? 1 : 0;
}
