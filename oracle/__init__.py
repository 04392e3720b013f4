"""CPU oracle for MergeShuffle: test infrastructure only (tests/, smoke(), bench cpu_baseline)."""
