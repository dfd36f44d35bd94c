// run_lshade_rs.hip -- the fused run kernels of L-SHADE-Restart, one per
// (k-step class, placement, team).
#include "run_kernel.h"

namespace sevo {

RunKernel run_table_lshade_rs(int ks, bool onchip, bool wave)
{
    return family_table<FAM_LSHADE_RS>(ks, onchip, wave);
}

}  // namespace sevo
