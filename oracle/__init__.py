"""FP64 CPU oracle for the LABFM hot path: test infrastructure only.

Only the tests, the smoke check and the benchmark's CPU-baseline leg may use
this package; the product library never imports it."""
