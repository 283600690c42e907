"""MI355X-native TFHE gate bootstrapping for location-based PIR (VeLoPIR, arXiv 2506.12761)."""
