// run_pso.hip -- the fused run kernels of PSO (global-best or ring, inertia or spherical), one per (k-step
// class, placement, team).
#include "run_kernel.h"

namespace sevo {

RunKernel run_table_pso(int ks, bool onchip, bool wave) { return family_table<FAM_PSO>(ks, onchip, wave); }

}  // namespace sevo
