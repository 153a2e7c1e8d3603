"""Seeded synthetic inputs (single-particle G buffers, signs) and workload shapes."""
from .hubbard import (C1_TINY, C2_PLAIN, C3_BATCHED, C4_RING, C5_SPLIT, PH_CHARGE,
                      PH_MAGNETIC, PP_UPDOWN, WORKLOADS, Workload, expansion_configs, g0_diag, g_elements,
                      g_matrices, noise_elements, signs)
