"""CPU oracle of the interpolation compressor: test infrastructure only.

Only the tests, the smoke check and the benchmark's CPU-baseline leg import this
package. It loads ``liboracle.so`` (plain single-threaded C, built from
``hiz_oracle.c``) and shares nothing with the GPU library.
"""
from .oracle import *  # noqa: F401,F403
