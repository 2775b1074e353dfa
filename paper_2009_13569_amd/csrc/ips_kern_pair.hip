// Kernel instantiations for element type pair.
#include "ips_kern_impl.hpp"

namespace ips {
const Launchers* launchers_pair() { return LaunchImpl<TPair>::table(); }
}  // namespace ips
