// Subdomain relaxation (filled in below).
#include "common.hpp"

namespace cd {
size_t relax_workspace_bytes(int op, int64_t n, int32_t n_patches, int64_t total_active,
                             int precision) {
  (void)op; (void)n; (void)n_patches; (void)total_active; (void)precision;
  return 0;
}
}  // namespace cd
