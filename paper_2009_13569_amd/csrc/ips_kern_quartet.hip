// Kernel instantiations for the Quartet (three u64 key words and a u64 value).
#include "ips_kern_impl.hpp"

namespace ips {
const Launchers* launchers_quartet() { return LaunchImpl<TQuartet>::table(); }
}  // namespace ips
