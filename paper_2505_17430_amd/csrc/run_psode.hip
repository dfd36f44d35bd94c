// run_psode.hip -- the fused run kernels of PSODE (PSO and SHADE halves with
// pairwise/3 selection), one per (k-step class, placement, team).
#include "run_kernel.h"

namespace sevo {

RunKernel run_table_psode(int ks, bool onchip, bool wave) { return family_table<FAM_PSODE>(ks, onchip, wave); }

}  // namespace sevo
