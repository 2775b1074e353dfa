// Kernel instantiations for element type u64.
#include "ips_kern_impl.hpp"

namespace ips {
const Launchers* launchers_u64() { return LaunchImpl<TU64>::table(); }
}  // namespace ips
