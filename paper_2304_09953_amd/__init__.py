"""MI355X-native rigid-receptor docking screen (LIGATE hot path)."""
