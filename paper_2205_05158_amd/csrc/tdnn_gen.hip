// Generic shapes of the tuned TDNN kernels (Sec. III-C network): compiled once per
// precision (DPD_GEN_PREC) and padded width (DPD_GEN_HP, 32, 64 or 128) for 8, 16 and
// 32 taps and 1..4 hidden layers.  The tap count and width of the model come at run
// time; the build names the unit's entry point through DPD_GEN_FN.
#include "tdnn_kernels.hpp"

#if !defined(DPD_GEN_PREC) || !defined(DPD_GEN_HP) || !defined(DPD_GEN_FN)
#error "tdnn_gen.hip is compiled with DPD_GEN_PREC, DPD_GEN_HP and DPD_GEN_FN defined"
#endif

namespace dpdmi {

const TdnnKernels* DPD_GEN_FN(int tp, int nl) {
  auto pick = [&]<int TP>() -> const TdnnKernels* {
    switch (nl) {
      case 1: return &TdnnShape<DPD_GEN_PREC, TP, DPD_GEN_HP, 1, true>::table;
      case 2: return &TdnnShape<DPD_GEN_PREC, TP, DPD_GEN_HP, 2, true>::table;
      case 3: return &TdnnShape<DPD_GEN_PREC, TP, DPD_GEN_HP, 3, true>::table;
      case 4: return &TdnnShape<DPD_GEN_PREC, TP, DPD_GEN_HP, 4, true>::table;
      default: return nullptr;
    }
  };
  if (tp == 8) return pick.template operator()<8>();
  if (tp == 16) return pick.template operator()<16>();
  if (tp == 32) return pick.template operator()<32>();
  return nullptr;
}

}  // namespace dpdmi
