"""FP64 CPU oracle for GCR / GCRV.  Test infrastructure only: imported by the
tests, the smoke check and the benchmark's CPU-baseline leg, never by the
library's product path."""
