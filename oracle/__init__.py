"""CPU oracle for the encrypted sparse matrix product -- TEST INFRASTRUCTURE ONLY.

Only the test suite, the smoke check and the benchmark's CPU-baseline leg may
import this package.  The GPU library does not, and shares no code with it.
"""
