"""MI355X-native FR-SG hot path (placeholder; binding added with the library)."""
