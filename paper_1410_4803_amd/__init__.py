"""pg -- pairwise genotype statistics (IBS matrices, LD windows) on AMD
MI355X, behind the C ABI of libpg.so (include/pg.h).

The statistics are those PLINK 1.9 accelerates with bit-parallel popcounts
(Chang et al., "Second-generation PLINK", arXiv 1410.4803): identity-by-state
counts per sample pair (section "Bitwise parallelism") and LD sums and r^2 per
variant pair (section "Bit population count"), and the greedy LD pruning
built on them (section "Linkage disequilibrium-based variant pruning"), and
the genomic relationship matrix (section "Partial sum lookup"), and the IBS
distance with complete-linkage clustering, the IBS similarity and the IBD
report by the method of moments (section "Identity-by-state matrices,
complete linkage clustering"; Table 2).  All computation runs in the
library's HIP kernels; this package only marshals arguments.
"""
from ._native import (LD_PAIR, PATHS, LAYOUTS, PgError, load as load_library,  # noqa: F401
                      last_error, status_str)
from .api import (Cohort, ibs_matrix, ibs_workspace_bytes, ibs_output_size,  # noqa: F401
                  ld_window, ld_workspace_bytes, ld_records, records_to_numpy, ld_prune,
                  prune_workspace_bytes, grm_matrix, grm_workspace_bytes, ibs_distance,
                  ibs_cluster, cluster_workspace_bytes, merges_to_numpy, peak_rates,
                  ibs_similarity, ibs_genome, genome_workspace_bytes, ibs_matrix_noalloc,
                  noalloc_scratch_bytes, resolve_path)
from .batch import Batch, IbsProblem, LdProblem  # noqa: F401
from .tune import Tuner  # noqa: F401

__all__ = ["Cohort", "ibs_matrix", "ibs_workspace_bytes", "ibs_output_size", "ld_window",
           "ld_workspace_bytes", "ld_records", "records_to_numpy", "LD_PAIR", "PATHS",
           "LAYOUTS", "PgError", "load_library", "last_error", "status_str", "Batch",
           "IbsProblem", "LdProblem", "Tuner", "ld_prune", "prune_workspace_bytes", "grm_matrix",
           "grm_workspace_bytes", "ibs_distance", "ibs_cluster", "cluster_workspace_bytes",
           "merges_to_numpy", "peak_rates", "ibs_similarity", "ibs_genome",
           "genome_workspace_bytes", "ibs_matrix_noalloc", "noalloc_scratch_bytes", "resolve_path"]
