// Kernel instantiations for element type rec100.
#include "ips_kern_impl.hpp"

namespace ips {
const Launchers* launchers_rec100() { return LaunchImpl<TRec100>::table(); }
}  // namespace ips
