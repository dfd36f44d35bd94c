// run_lshade.hip -- the fused run kernels of L-SHADE, one per (k-step
// class, placement, team).
#include "run_kernel.h"

namespace sevo {

RunKernel run_table_lshade(int ks, bool onchip, bool wave) { return family_table<FAM_LSHADE>(ks, onchip, wave); }

}  // namespace sevo
