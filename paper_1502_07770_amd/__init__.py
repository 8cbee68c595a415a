"""MI355X-native batched TV-chain prox and 2D TV (placeholder, binding follows)."""
