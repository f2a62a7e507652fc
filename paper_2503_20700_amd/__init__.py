"""MI355X-native spin-adapted two-site DMRG hot path (H*psi, Davidson,
truncation, operator-block renormalisation) behind a C ABI; see include/dmrg.h."""
from .binding import BF16, FP32, FP64, DMRG, DMRGError, load  # noqa: F401
