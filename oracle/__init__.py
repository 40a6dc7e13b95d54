"""FP64 CPU oracle for the aggregation-AMG method (test infrastructure only).

Imported by the tests, the smoke check and the benchmark's CPU-baseline leg;
never by the product path."""
