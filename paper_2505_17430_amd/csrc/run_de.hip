// run_de.hip -- the fused run kernels of DE rand/1/bin, one per (k-step
// class, placement, team).
#include "run_kernel.h"

namespace sevo {

RunKernel run_table_de(int ks, bool onchip, bool wave) { return family_table<FAM_DE>(ks, onchip, wave); }

}  // namespace sevo
