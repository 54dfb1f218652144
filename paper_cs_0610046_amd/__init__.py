"""MI355X-native running max-min filter (placeholder; the binding is loaded lazily)."""
