// Kernel instantiation for one species count (compiled once per CSI_NS).
#include "csi_runner.hpp"

#ifndef CSI_NS
#error "CSI_NS must be defined"
#endif
#define CSI_CAT2(a, b) a##b
#define CSI_CAT(a, b) CSI_CAT2(a, b)

csi::IRunner *CSI_CAT(csi_make_runner_, CSI_NS)(int nt) {
  if (nt == 1) return new csi::Runner<CSI_NS, 1>();
  return new csi::Runner<CSI_NS, 2>();
}
