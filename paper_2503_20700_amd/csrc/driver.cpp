// Davidson eigensolver and truncation at the two-site block.
#include <string>

#include "../../include/dmrg.h"
#include "session.hpp"

extern "C" int dmrg_davidson_step(dmrg_ctx*, int, double*, double*, double*, int*, int*) { return DMRG_ERR_ARG; }
extern "C" int dmrg_truncate(dmrg_ctx*, int, const double*, int, int, double, double*, int*) { return DMRG_ERR_ARG; }
extern "C" int dmrg_cut_spectrum(dmrg_ctx*, double*, int*, int*, int) { return DMRG_ERR_ARG; }
