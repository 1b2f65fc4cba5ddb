"""FP64 CPU oracle of the free-surface LBM foaming step (test infrastructure only).

Only the tests, the smoke check and the benchmark's CPU-baseline leg import this
package. The GPU library never does.
"""
from .oracle import Oracle, load_library  # noqa: F401
