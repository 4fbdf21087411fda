"""MI355X-native near-field force (arXiv:1810.02916)."""
