"""CPU oracle for the TFHE bootstrapping path (test infrastructure only)."""
