// run_shade.hip -- the fused run kernels of SHADE, one per (k-step
// class, placement, team).
#include "run_kernel.h"

namespace sevo {

RunKernel run_table_shade(int ks, bool onchip, bool wave) { return family_table<FAM_SHADE>(ks, onchip, wave); }

}  // namespace sevo
