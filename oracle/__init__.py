"""FP64 CPU oracle for SP2 density-matrix purification (test infrastructure).

This package is test infrastructure only. It is imported by the tests, by the
smoke check and by the CPU-baseline leg of the benchmark, never by the
library or its Python binding. It shares no code with the GPU path: it is a
plain, slow, step-by-step restatement of the paper's algorithm in NumPy
float64 (Kruchinina, Rudberg, Rubensson, "Parameterless stopping criteria
for recursive density matrix expansions", Alg. 2 and sec. 2; SP2-ACC,
Alg. 3 and Alg. 4; McWeeny and McW-ACC, sec. 3).
"""
from .sp2 import (  # noqa: F401
    C_SP2,
    Q_TILDE,
    SP2Result,
    Status,
    f0,
    truncate,
    choose_polynomial,
    stop_fires,
    observed_order,
    sp2,
    density_from_eigenvectors,
    density_from_eigh,
    g_ratio,
    p_sp1,
    p_sp2,
    mixed_norm,
)
from .sp2acc import (  # noqa: F401
    EPS_M,
    DELTA,
    Schedule,
    bounds_valid,
    acc_schedule,
    acc_polynomial,
    sp2_acc,
)
from .mcweeny import (  # noqa: F401
    C_MW,
    p_mw,
    f0_mw,
    mw_gamma,
    mwa_alpha,
    p_mwa,
    mcweeny,
)
