// (serving loop: added later)
