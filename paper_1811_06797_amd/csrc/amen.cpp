// Block-AMEn solver (placeholder until the sweep lands).
#include "common.hpp"
namespace iga {
int amen_impl(iga_ctx*, const iga_kkt*, const iga_tt*, double, const iga_amen_opts*, const iga_btt*,
              iga_btt**, iga_amen_stats*) {
  fail(IGA_EINVAL, "amen_solve: not built yet");
}
}  // namespace iga
