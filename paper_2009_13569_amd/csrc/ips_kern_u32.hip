// Kernel instantiations for element type u32.
#include "ips_kern_impl.hpp"

namespace ips {
const Launchers* launchers_u32() { return LaunchImpl<TU32>::table(); }
}  // namespace ips
