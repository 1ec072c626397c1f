"""MI355X-native separable N-point correlation function estimator
(Philcox & Slepian, arXiv:2106.10278): HIP kernels for gfx950 behind the C
ABI of include/npcf.h, with a thin ctypes binding (:mod:`.binding`).

The HIP library is loaded lazily on first use; importing the package never
touches the GPU.
"""
from .binding import NPCF, NPCFError, NPCFLibraryMissing, load_library, stored_state_labels, stored_states  # noqa: F401
