"""CPU FP64 oracle: test infrastructure only.

Only the tests, the smoke check and the benchmark's CPU-baseline leg may
import this package.  It shares no code with the HIP library
(``paper_2103_10975_amd``) and imports nothing from it.
"""
