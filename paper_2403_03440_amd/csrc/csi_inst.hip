// Kernel instantiation for one species count and temperature model (compiled
// once per (CSI_NS, CSI_NT)).
#include "csi_runner.hpp"

#if !defined(CSI_NS) || !defined(CSI_NT)
#error "CSI_NS and CSI_NT must be defined"
#endif
#define CSI_CAT4(a, b, c, d) a##b##c##d
#define CSI_FACTORY(ns, nt) CSI_CAT4(csi_make_runner_, ns, _, nt)

csi::IRunner *CSI_FACTORY(CSI_NS, CSI_NT)() { return new csi::Runner<CSI_NS, CSI_NT>(); }
