"""FP64 CPU oracle for the SRM EM sweep -- test infrastructure only.

Only the test-suite, the smoke check and the benchmark's CPU-baseline leg may
import this package.  The device library never calls it and shares no code
with it.
"""
from .srm_oracle import (  # noqa: F401
    OracleRankError, OracleNotPD, demean, zscore, posterior, loglik, polar_svd,
    m_step_subject, em_fit, naive_estep, fit_gram, gram_summary,
    fit_gram_summaries, w_of, philox4x64, seeded_gaussian,
    seeded_start,
)
