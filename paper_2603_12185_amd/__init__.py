"""MI355X-native complementarity-free contact step (C-ABI library + thin binding)."""
