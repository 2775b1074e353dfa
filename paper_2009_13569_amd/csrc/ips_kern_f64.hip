// Kernel instantiations for element type f64.
#include "ips_kern_impl.hpp"

namespace ips {
const Launchers* launchers_f64() { return LaunchImpl<TF64>::table(); }
}  // namespace ips
