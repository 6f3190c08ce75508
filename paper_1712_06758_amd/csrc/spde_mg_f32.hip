// Multigrid kernels and their launchers with float levels (a translation unit of
// its own, so that the two precisions compile in parallel).
#define SPDE_MG_T float
#define SPDE_MG_NAME f32
#include "spde_mg.inc"
#include "spde_vcycle.inc"
#include "spde_mg_launch.inc"
