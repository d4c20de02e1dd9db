"""Hybrid-dealiased real convolution for MI355X (placeholder; binding comes with the library)."""
