// Multigrid kernels and their launchers with double levels (a translation unit of
// its own, so that the two precisions compile in parallel).
#define SPDE_MG_T double
#define SPDE_MG_NAME f64
#include "spde_mg.inc"
#include "spde_vcycle.inc"
#include "spde_mg_launch.inc"
