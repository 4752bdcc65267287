"""FP64 CPU oracle for coded QR.  Test infrastructure only: imported by the
test suite, the smoke check and the benchmark's CPU-baseline leg, never by the
library path."""
