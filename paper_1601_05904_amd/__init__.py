"""AIDW with even-grid kNN on MI355X (placeholder; binding added with the library)."""
