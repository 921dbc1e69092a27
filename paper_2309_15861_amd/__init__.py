"""MI355X-native optical-photon pipeline (arXiv:2309.15861 hot path)."""
